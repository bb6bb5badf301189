/* Drives every public call of the D2Q9 and D3Q19 oracles over small
 * lattices (all bases, both inits, sampling, structure factors, error
 * paths), for a build under the address and undefined-behaviour sanitizers
 * (tests/test_oracle_sanitizers.py).  Prints "ok" and exits 0 when every
 * call returned what it should; the sanitizers abort on any memory or
 * undefined-behaviour fault. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "flbref.h"
#include "flbref3.h"

static int fails = 0;
#define CHECK(cond)                                                     \
  do {                                                                  \
    if (!(cond)) {                                                      \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++fails;                                                          \
    }                                                                   \
  } while (0)

static void d2q9_site_calls(void) {
  int32_t vx[9], vy[9];
  double w[9], m[81], mt[81], ug[2], N[6], f[9], fo[9];
  flbref_velocities(vx, vy, w);
  flbref_hermite_matrix(m);
  for (int i = 0; i < 9; ++i) f[i] = flbref_equilibrium(i, 1.1, 0.1, -0.05);
  CHECK(flbref_fnorm_basis(0.1, -0.05, mt) == FLBREF_OK);
  CHECK(flbref_fnorm_basis(0.5, 0.5, mt) == FLBREF_E_INVALID_VELOCITY);
  CHECK(flbref_lut_basis(0.013, -0.027, mt, ug) == FLBREF_OK);
  CHECK(flbref_lut_basis(0.9, 0.0, mt, ug) != FLBREF_OK);
  const uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6};
  uint32_t out[4];
  flbref_philox4x32_10(ctr, key, out);
  flbref_site_gaussians(7, 11, 13, 0, N);
  flbref_params p;
  memset(&p, 0, sizeof(p));
  p.nx = p.ny = 4;
  p.rho0 = 1.0;
  p.kT = 1e-4;
  for (int a = 0; a < 6; ++a) p.tau[a] = 0.7 + 0.1 * a;
  p.seed = 3;
  for (int b = 0; b < 3; ++b) {
    p.basis = b;
    CHECK(flbref_collide(&p, f, 5, 9, fo) == FLBREF_OK);
  }
  p.basis = FLBREF_BASIS_FNORM_LUT;
  CHECK(flbref_collide_lut_at(&p, f, 5, 9, 5, -2, fo) == FLBREF_OK);
  CHECK(flbref_collide_lut_at(&p, f, 5, 9, 26, 0, fo) == FLBREF_E_INVALID_VELOCITY);
  p.basis = FLBREF_BASIS_HERMITE;
  CHECK(flbref_collide_lut_at(&p, f, 5, 9, 0, 0, fo) == FLBREF_E_ARG);
  double bad[9];
  for (int i = 0; i < 9; ++i) bad[i] = flbref_equilibrium(i, 1.0, 0.9, 0.0);
  p.basis = FLBREF_BASIS_FNORM_LOCAL;
  CHECK(flbref_collide(&p, bad, 0, 0, fo) == FLBREF_E_INVALID_VELOCITY);
}

static void d2q9_lattice(int basis, int init, int nx, int ny) {
  flbref_params p;
  memset(&p, 0, sizeof(p));
  p.nx = nx;
  p.ny = ny;
  p.rho0 = 1.0;
  p.ux0 = 0.08;
  p.uy0 = -0.03;
  p.kT = 1e-4;
  for (int a = 0; a < 6; ++a) p.tau[a] = 0.6 + 0.15 * a;
  p.seed = 9;
  p.basis = basis;
  p.init = init;
  p.sample_every = 1;
  p.sk_every = 3;
  p.block_steps = 4;
  flbref_lattice* L = NULL;
  CHECK(flbref_lattice_create(&p, &L) == FLBREF_OK);
  if (!L) return;
  const size_t n = (size_t)nx * ny;
  double* f = malloc(9 * n * sizeof(double));
  double* g = malloc(9 * n * sizeof(double));
  double* r = malloc(3 * n * sizeof(double));
  if (init == FLBREF_INIT_FIELDS) {
    for (size_t s = 0; s < n; ++s) {
      r[s] = 1.0 + 0.01 * sin((double)s);
      r[n + s] = 0.08 + 0.01 * cos((double)s);
      r[2 * n + s] = -0.03;
    }
    CHECK(flbref_lattice_set_fields(L, r, r + n, r + 2 * n) == FLBREF_OK);
  }
  CHECK(flbref_lattice_step(L, 7) == FLBREF_OK);
  CHECK(flbref_lattice_time(L) == 7);
  CHECK(flbref_lattice_read_populations(L, f) == FLBREF_OK);
  for (int at = 0; at < 3; ++at) CHECK(flbref_lattice_read_moments(L, at, g) == FLBREF_OK);
  CHECK(flbref_lattice_read_moments(L, 7, g) == FLBREF_E_ARG);
  flbref_cov c;
  CHECK(flbref_lattice_read_covariance(L, &c) == FLBREF_OK);
  CHECK(c.nsamples == 7 * n && isfinite(c.cov_f[0]));
  for (int wh = 0; wh < 5; ++wh)
    CHECK(flbref_lattice_read_structure_factor(L, wh, g) == FLBREF_OK);
  double mode[2];
  CHECK(flbref_lattice_read_fourier_mode(L, 2, 1, 0, mode) == FLBREF_OK);
  CHECK(flbref_lattice_reset_stats(L) == FLBREF_OK);
  CHECK(flbref_lattice_set_populations(L, f, 8) == FLBREF_OK);
  CHECK(flbref_lattice_step(L, 2) == FLBREF_OK);
  CHECK(flbref_lattice_error_step(L) == -1);
  /* a site outside the validity region stops the step and records it (the
   * Hermite basis needs no f-norm and steps on) */
  for (int i = 0; i < 9; ++i) f[i * n] = flbref_equilibrium(i, 1.0, 0.9, 0.0);
  CHECK(flbref_lattice_set_populations(L, f, 20) == FLBREF_OK);
  const int want = basis == FLBREF_BASIS_HERMITE ? FLBREF_OK : FLBREF_E_INVALID_VELOCITY;
  CHECK(flbref_lattice_step(L, 1) == want);
  CHECK(flbref_lattice_error_step(L) == (want == FLBREF_OK ? -1 : 20));
  flbref_lattice_destroy(L);
  free(f);
  free(g);
  free(r);
}

static void d3q19_calls(int basis) {
  int32_t vx[19], vy[19], vz[19];
  double w[19], m[361], mt[361], N[15], f[19], fo[19];
  flbref3_velocities(vx, vy, vz, w);
  flbref3_basis(m);
  CHECK(flbref3_fnorm_basis(0.05, -0.02, 0.03, mt) == FLBREF_OK);
  flbref3_site_gaussians(3, 4, 5, 0, N);
  for (int i = 0; i < 19; ++i) f[i] = flbref3_equilibrium(i, 1.0, 0.05, -0.02, 0.03);
  flbref3_params p;
  memset(&p, 0, sizeof(p));
  p.nx = 3;
  p.ny = 4;
  p.nz = 5;
  p.basis = basis;
  p.rho0 = 1.0;
  p.ux0 = 0.05;
  p.kT = 1e-4;
  for (int a = 0; a < 15; ++a) p.tau[a] = 0.6 + 0.05 * a;
  p.seed = 2;
  p.sample_every = 1;
  p.block_steps = 2;
  CHECK(flbref3_collide(&p, f, 1, 2, fo) == FLBREF_OK);
  flbref3_lattice* L = NULL;
  CHECK(flbref3_lattice_create(&p, &L) == FLBREF_OK);
  if (!L) return;
  const size_t n = 3 * 4 * 5;
  double* buf = malloc(19 * n * sizeof(double));
  CHECK(flbref3_lattice_step(L, 5) == FLBREF_OK);
  CHECK(flbref3_lattice_time(L) == 5);
  CHECK(flbref3_lattice_read_populations(L, buf) == FLBREF_OK);
  flbref3_cov c;
  CHECK(flbref3_lattice_read_covariance(L, &c) == FLBREF_OK);
  CHECK(c.nsamples == 5 * n);
  CHECK(flbref3_lattice_reset_stats(L) == FLBREF_OK);
  CHECK(flbref3_lattice_set_populations(L, buf, 6) == FLBREF_OK);
  CHECK(flbref3_lattice_step(L, 2) == FLBREF_OK);
  flbref3_lattice_destroy(L);
  free(buf);
}

int main(void) {
  d2q9_site_calls();
  flbref_set_threads(3);
  d2q9_lattice(FLBREF_BASIS_FNORM_LOCAL, FLBREF_INIT_THERMAL, 8, 6);
  flbref_set_threads(1);
  for (int b = 0; b < 3; ++b)
    for (int init = 0; init < 3; ++init) {
      d2q9_lattice(b, init, 8, 4);
      d2q9_lattice(b, init, 5, 3);  /* odd sides: direct DFTs */
    }
  d3q19_calls(FLBREF3_BASIS_FNORM_LOCAL);
  d3q19_calls(FLBREF3_BASIS_HERMITE);
  if (fails) {
    fprintf(stderr, "%d checks failed\n", fails);
    return 1;
  }
  printf("ok\n");
  return 0;
}
