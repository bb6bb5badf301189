/*
 * flbref3 — plain FP64 CPU oracle for a D3Q19 form of the fluctuating
 * lattice-Boltzmann step in the velocity-dependent f-norm basis (Kaehler &
 * Wagner; the paper works in D2Q9 and states that the construction carries
 * over to other velocity sets, Sec. V).
 *
 * TEST INFRASTRUCTURE ONLY, like flbref.h: nothing in the product library
 * includes, links or calls it, and it shares no source with the GPU code.
 *
 * The D3Q19 model is this oracle's own reading of that generalisation:
 *   velocities: rest, the six (+-1,0,0)..., the twelve (+-1,+-1,0)...,
 *     opposite pairs adjacent (1,2), (3,4), ...; weights 1/3, 1/18, 1/36;
 *   equilibrium f^0_i(rho,u) = w_i rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u^2)
 *     (the form of eq. (A1));
 *   the "Hermite" rows m^a: Gram-Schmidt under the weights w of the
 *     polynomials 1; v_x, v_y, v_z; v_x v_y, v_x v_z, v_y v_z, v_x^2 - v_y^2,
 *     v_x^2 + v_y^2 - 2 v_z^2, v^2; v_x (v_y^2 + v_z^2), v_y (v_x^2 + v_z^2),
 *     v_z (v_x^2 + v_y^2), v_x (v_y^2 - v_z^2), v_y (v_z^2 - v_x^2),
 *     v_z (v_x^2 - v_y^2); v^4, (2 v_x^2 - v_y^2 - v_z^2) v^2,
 *     (v_y^2 - v_z^2) v^2 (orthonormal under w, like the table of eq. (A3));
 *   the f-norm rows m~^a: the same Gram-Schmidt of those rows under
 *     g = f^0(1, u) (eqs. (27)-(30));
 *   15 non-conserved modes a = 4..18, each relaxed with its own tau and
 *     given noise of amplitude sqrt(mu rho (2 tau - 1)) / tau (eq. (20));
 *   noise: four Philox4x32-10 blocks per site and step, counter (site, c,
 *     step lo, step hi XOR tag) for c = 0..3, key = seed; sixteen 24-bit
 *     integers (top 24 bits of each word, block by block), uniforms
 *     (U + 1/2) 2^-24, Box-Muller on consecutive pairs; the first fifteen
 *     Gaussians drive modes 4..18.
 */
#ifndef FLBREF3_H
#define FLBREF3_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { FLBREF3_BASIS_FNORM_LOCAL = 0, FLBREF3_BASIS_HERMITE = 1 };

typedef struct {
  int32_t nx, ny, nz;
  int32_t basis;
  double rho0, ux0, uy0, uz0;
  double kT;          /* mu = 3 kT */
  double tau[15];     /* modes a = 4..18 */
  uint64_t seed;
  int32_t sample_every;
  int32_t block_steps;
} flbref3_params;

typedef struct {
  uint64_t nsamples, nblocks;
  double mean_df[19];   /* <f_i> - f_i^0(rho0, u0)            */
  double cov_f[361];    /* <df_i df_j>, empirical-mean centred */
  double se_cov_f[361]; /* time-block standard errors          */
} flbref3_cov;

typedef struct flbref3_lattice flbref3_lattice;

void flbref3_velocities(int32_t vx[19], int32_t vy[19], int32_t vz[19], double w[19]);
void flbref3_basis(double m[361]);                 /* row a, column i */
double flbref3_equilibrium(int i, double rho, double ux, double uy, double uz);
int flbref3_fnorm_basis(double ux, double uy, double uz, double mt[361]);
void flbref3_site_gaussians(uint64_t seed, uint64_t site, uint64_t step, uint32_t tag,
                            double N[15]);
int flbref3_collide(const flbref3_params* p, const double f[19], uint64_t site, uint64_t step,
                    double fout[19]);

int flbref3_lattice_create(const flbref3_params* p, flbref3_lattice** out);
int flbref3_lattice_set_populations(flbref3_lattice* L, const double* f, uint64_t t);
int flbref3_lattice_step(flbref3_lattice* L, uint64_t nsteps);
int flbref3_lattice_read_populations(flbref3_lattice* L, double* f);  /* [19][nz][ny][nx] */
int flbref3_lattice_read_covariance(flbref3_lattice* L, flbref3_cov* out);
int flbref3_lattice_reset_stats(flbref3_lattice* L);
uint64_t flbref3_lattice_time(flbref3_lattice* L);
void flbref3_lattice_destroy(flbref3_lattice* L);

#ifdef __cplusplus
}
#endif
#endif
