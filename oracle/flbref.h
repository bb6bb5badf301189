/*
 * flbref — plain FP64 CPU oracle for the fluctuating D2Q9 lattice Boltzmann
 * step in the velocity-dependent f-norm basis (Kaehler & Wagner, "A
 * fluctuating lattice-Boltzmann method with improved Galilean invariance").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this code; only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg use it.  It shares no source with the GPU
 * library: constants, tables, the counter-based generator and the
 * Gram-Schmidt construction are all written out again here.
 *
 * Every routine follows the paper literally and slowly: per-site classical
 * Gram-Schmidt (Sec. IV, eqs. (27)-(32)), collision in moment space
 * (Sec. II, eq. (6)), noise amplitude from the fluctuation-dissipation
 * relation (eq. (20)), streaming (eq. (1)), correlators (eqs. (16), (23),
 * (34)) and structure factors (eqs. (24)-(26)).
 */
#ifndef FLBREF_H
#define FLBREF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  FLBREF_OK = 0,
  FLBREF_E_ARG = -1,
  FLBREF_E_OOM = -2,
  FLBREF_E_INVALID_VELOCITY = -4,
  FLBREF_E_NONFINITE = -5
};

enum { FLBREF_BASIS_FNORM_LOCAL = 0, FLBREF_BASIS_HERMITE = 1, FLBREF_BASIS_FNORM_LUT = 2 };
enum { FLBREF_INIT_EQUILIBRIUM = 0, FLBREF_INIT_THERMAL = 1, FLBREF_INIT_FIELDS = 2 };

/* Same field layout as the GPU library's parameter block (written out
 * separately on purpose). */
typedef struct {
  int32_t nx, ny;
  double rho0, ux0, uy0;
  double kT;          /* noise strength mu = 3 kT multiplies every xi^a^2 */
  double tau[6];      /* modes a = 3..8: Pi_xx-yy, Pi_xy, Pi_xx+yy, q_x, q_y, eps */
  uint64_t seed;
  int32_t precision;  /* ignored by the oracle: it always computes in FP64 */
  int32_t basis;
  int32_t init;
  int32_t sample_every;
  int32_t sk_every;
  int32_t block_steps;
} flbref_params;

typedef struct {
  uint64_t nsamples;      /* number of (site, time) samples            */
  uint64_t nblocks;       /* number of closed time blocks               */
  double mean_df[9];      /* <f_i> - f_i^0(rho0, u0)                    */
  double cov_f[81];       /* <df_i df_j>, empirical-mean centred        */
  double cov_m_fnorm_u0[81]; /* m~(u0) C m~(u0)^T                        */
  double cov_m_hermite[81];  /* m C m^T                                  */
  double se_cov_f[81];
  double se_cov_m[81];
} flbref_cov;

typedef struct flbref_lattice flbref_lattice;

/* ---- single-site building blocks (exported for the pins) ---- */
void flbref_velocities(int32_t vx[9], int32_t vy[9], double w[9]);
void flbref_hermite_matrix(double m[81]);                       /* eq. (A3), row a, column i */
double flbref_equilibrium(int i, double rho, double ux, double uy); /* eq. (A1)              */
int flbref_fnorm_basis(double ux, double uy, double mt[81]);    /* eqs. (27)-(30)             */
void flbref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void flbref_site_gaussians(uint64_t seed, uint64_t site, uint64_t step, uint32_t tag, double N[6]);
int flbref_collide(const flbref_params* p, const double f[9], uint64_t site, uint64_t step,
                   double fout[9]);
int flbref_lut_basis(double ux, double uy, double mt[81], double ug[2]);
/* Table-variant collision at grid point (ix, iy) * 0.02, |ix|, |iy| <= 25. */
int flbref_collide_lut_at(const flbref_params* p, const double f[9], uint64_t site,
                          uint64_t step, int32_t ix, int32_t iy, double fout[9]);

/* ---- lattice ---- */
/* Threads of the lattice calls' per-site loops (default 1; results are the
 * same for any count). */
void flbref_set_threads(int n);
int flbref_lattice_create(const flbref_params* p, flbref_lattice** out);
int flbref_lattice_set_fields(flbref_lattice* L, const double* rho, const double* ux,
                              const double* uy);
int flbref_lattice_set_populations(flbref_lattice* L, const double* f9xy, uint64_t t);
int flbref_lattice_step(flbref_lattice* L, uint64_t nsteps);
int flbref_lattice_read_populations(flbref_lattice* L, double* f9xy);
int flbref_lattice_read_moments(flbref_lattice* L, int32_t at, double* m9xy);
int flbref_lattice_read_covariance(flbref_lattice* L, flbref_cov* out);
int flbref_lattice_read_structure_factor(flbref_lattice* L, int32_t which, double* out_xy);
int flbref_lattice_read_fourier_mode(flbref_lattice* L, int32_t which, int32_t kx, int32_t ky,
                                     double out[2]);
int flbref_lattice_reset_stats(flbref_lattice* L);
uint64_t flbref_lattice_time(flbref_lattice* L);
int64_t flbref_lattice_error_step(flbref_lattice* L);
void flbref_lattice_destroy(flbref_lattice* L);

#ifdef __cplusplus
}
#endif
#endif
