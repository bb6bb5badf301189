/*
 * flbref3.c — the D3Q19 oracle declared in flbref3.h (test infrastructure
 * only).  Plain, slow FP64 C: every collision builds its basis by classical
 * Gram-Schmidt, exactly as the D2Q9 oracle does (Sec. IV, eqs. (27)-(32)),
 * then relaxes and adds noise in that basis (Sec. II, eq. (6), eq. (20)).
 */
#include "flbref3.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "flbref.h"

#define Q 19

static const int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

static double weight(int i) { return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0); }

void flbref3_velocities(int32_t vx[19], int32_t vy[19], int32_t vz[19], double w[19]) {
  for (int i = 0; i < Q; ++i) {
    vx[i] = CX[i];
    vy[i] = CY[i];
    vz[i] = CZ[i];
    w[i] = weight(i);
  }
}

/* The 19 start polynomials, in order, evaluated at velocity i. */
static double poly(int a, int i) {
  const double x = CX[i], y = CY[i], z = CZ[i];
  const double x2 = x * x, y2 = y * y, z2 = z * z, v2 = x2 + y2 + z2;
  switch (a) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return x * y;
    case 5: return x * z;
    case 6: return y * z;
    case 7: return x2 - y2;
    case 8: return x2 + y2 - 2.0 * z2;
    case 9: return v2;
    case 10: return x * (y2 + z2);
    case 11: return y * (x2 + z2);
    case 12: return z * (x2 + y2);
    case 13: return x * (y2 - z2);
    case 14: return y * (z2 - x2);
    case 15: return z * (x2 - y2);
    case 16: return v2 * v2;
    case 17: return (2.0 * x2 - y2 - z2) * v2;
    default: return (y2 - z2) * v2;
  }
}

/* Classical Gram-Schmidt of the rows src[a][i] under <a,b> = sum_i a_i k_i
 * b_i, positive normalisation by the square root of the norm.  Returns -1
 * if a vector degenerates. */
static int gram_schmidt(const double src[361], const double k[19], double out[361]) {
  for (int a = 0; a < Q; ++a) {
    double v[Q];
    for (int i = 0; i < Q; ++i) v[i] = src[a * Q + i];
    for (int b = 0; b < a; ++b) {
      double proj = 0.0;
      for (int i = 0; i < Q; ++i) proj += out[b * Q + i] * k[i] * src[a * Q + i];
      for (int i = 0; i < Q; ++i) v[i] -= proj * out[b * Q + i];
    }
    double nrm = 0.0;
    for (int i = 0; i < Q; ++i) nrm += v[i] * k[i] * v[i];
    if (!(nrm > 0.0)) return -1;
    const double s = 1.0 / sqrt(nrm);
    for (int i = 0; i < Q; ++i) out[a * Q + i] = v[i] * s;
  }
  return 0;
}

void flbref3_basis(double m[361]) {
  double p[361], w[Q];
  for (int a = 0; a < Q; ++a)
    for (int i = 0; i < Q; ++i) p[a * Q + i] = poly(a, i);
  for (int i = 0; i < Q; ++i) w[i] = weight(i);
  (void)gram_schmidt(p, w, m);
}

double flbref3_equilibrium(int i, double rho, double ux, double uy, double uz) {
  const double cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
  const double uu = ux * ux + uy * uy + uz * uz;
  return weight(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
}

int flbref3_fnorm_basis(double ux, double uy, double uz, double mt[361]) {
  double m[361], g[Q];
  flbref3_basis(m);
  for (int i = 0; i < Q; ++i) {
    g[i] = flbref3_equilibrium(i, 1.0, ux, uy, uz);
    if (!(g[i] > 0.0)) return FLBREF_E_INVALID_VELOCITY;
  }
  return gram_schmidt(m, g, mt) == 0 ? FLBREF_OK : FLBREF_E_INVALID_VELOCITY;
}

void flbref3_site_gaussians(uint64_t seed, uint64_t site, uint64_t step, uint32_t tag,
                            double N[15]) {
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t U[16];
  for (int c = 0; c < 4; ++c) {
    const uint32_t ctr[4] = {(uint32_t)site, (uint32_t)c, (uint32_t)step,
                             (uint32_t)(step >> 32) ^ tag};
    uint32_t w[4];
    flbref_philox4x32_10(ctr, key, w);
    for (int k = 0; k < 4; ++k) U[4 * c + k] = w[k] >> 8;
  }
  const double two_pi = 2.0 * 3.14159265358979323846;
  for (int p = 0; p < 8; ++p) {
    const double ua = ((double)U[2 * p] + 0.5) / 16777216.0;
    const double ub = ((double)U[2 * p + 1] + 0.5) / 16777216.0;
    const double r = sqrt(-2.0 * log(ua));
    if (2 * p < 15) N[2 * p] = r * cos(two_pi * ub);
    if (2 * p + 1 < 15) N[2 * p + 1] = r * sin(two_pi * ub);
  }
}

/* One collision: rho, u from f; the basis (f-norm: Gram-Schmidt under
 * g = f^0(1,u); Hermite: the fixed rows, with n = w m); moments M^a; for the
 * fifteen non-conserved modes M*^a = M^a - (M^a - M^{a,eq}) / tau^a + xi^a N
 * with M^{a,eq} = rho delta^{a0} in the f-norm and the moments of
 * f^0(rho, u) in the Hermite rows; f* = sum_a n^a M*^a. */
int flbref3_collide(const flbref3_params* p, const double f[19], uint64_t site, uint64_t step,
                    double fout[19]) {
  double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
  for (int i = 0; i < Q; ++i) {
    rho += f[i];
    jx += f[i] * CX[i];
    jy += f[i] * CY[i];
    jz += f[i] * CZ[i];
  }
  if (!(rho > 0.0) || !isfinite(jx) || !isfinite(jy) || !isfinite(jz)) return FLBREF_E_NONFINITE;
  const double ux = jx / rho, uy = jy / rho, uz = jz / rho;
  double m[361], k[Q], Meq[Q];
  if (p->basis == FLBREF3_BASIS_HERMITE) {
    flbref3_basis(m);
    for (int i = 0; i < Q; ++i) k[i] = weight(i);
    for (int a = 0; a < Q; ++a) {
      double s = 0.0;
      for (int i = 0; i < Q; ++i) s += m[a * Q + i] * flbref3_equilibrium(i, rho, ux, uy, uz);
      Meq[a] = s;
    }
  } else {
    const int rc = flbref3_fnorm_basis(ux, uy, uz, m);
    if (rc != FLBREF_OK) return rc;
    for (int i = 0; i < Q; ++i) k[i] = flbref3_equilibrium(i, 1.0, ux, uy, uz);
    for (int a = 0; a < Q; ++a) Meq[a] = a == 0 ? rho : 0.0;
  }
  double M[Q];
  for (int a = 0; a < Q; ++a) {
    double s = 0.0;
    for (int i = 0; i < Q; ++i) s += m[a * Q + i] * f[i];
    M[a] = s;
  }
  const double mu = 3.0 * p->kT;
  double N[15] = {0};
  if (mu > 0.0) flbref3_site_gaussians(p->seed, site, step, 0u, N);
  double dM[Q] = {0};
  for (int a = 4; a < Q; ++a) {
    const double tau = p->tau[a - 4];
    const double xi = sqrt(mu * rho * (2.0 * tau - 1.0)) / tau;
    dM[a] = -(M[a] - Meq[a]) / tau + xi * N[a - 4];
  }
  for (int i = 0; i < Q; ++i) {
    double s = 0.0;
    for (int a = 4; a < Q; ++a) s += m[a * Q + i] * k[i] * dM[a];
    fout[i] = f[i] + s;
  }
  return FLBREF_OK;
}

/* ------------------------------------------------------------- lattice */
struct flbref3_lattice {
  flbref3_params p;
  size_t N;
  double* f;     /* [19][N], the post-streaming (pre-collision) state */
  double* tmp;
  uint64_t t;
  /* correlator sums: 19 means + 190 products (i <= j), per time block */
  double open[209];
  uint64_t open_samples;
  double* blocks;
  uint64_t* block_samples;
  uint64_t nblocks, cap;
};

static size_t idx3(const flbref3_lattice* L, int x, int y, int z) {
  return ((size_t)z * L->p.ny + y) * L->p.nx + x;
}

int flbref3_lattice_create(const flbref3_params* p, flbref3_lattice** out) {
  *out = NULL;
  if (p->nx < 3 || p->ny < 3 || p->nz < 3 || !(p->rho0 > 0) || p->kT < 0)
    return FLBREF_E_ARG;
  for (int a = 0; a < 15; ++a)
    if (!(p->tau[a] > 0.5)) return FLBREF_E_ARG;
  flbref3_lattice* L = (flbref3_lattice*)calloc(1, sizeof(*L));
  if (!L) return FLBREF_E_OOM;
  L->p = *p;
  L->N = (size_t)p->nx * p->ny * p->nz;
  L->f = (double*)malloc(sizeof(double) * Q * L->N);
  L->tmp = (double*)malloc(sizeof(double) * Q * L->N);
  if (!L->f || !L->tmp) {
    flbref3_lattice_destroy(L);
    return FLBREF_E_OOM;
  }
  for (int i = 0; i < Q; ++i) {
    const double fe = flbref3_equilibrium(i, p->rho0, p->ux0, p->uy0, p->uz0);
    for (size_t s = 0; s < L->N; ++s) L->f[i * L->N + s] = fe;
  }
  *out = L;
  return FLBREF_OK;
}

int flbref3_lattice_set_populations(flbref3_lattice* L, const double* f, uint64_t t) {
  memcpy(L->f, f, sizeof(double) * Q * L->N);
  L->t = t;
  return FLBREF_OK;
}

static void close_block(flbref3_lattice* L) {
  if (L->open_samples == 0) return;
  if (L->nblocks == L->cap) {
    L->cap = L->cap ? 2 * L->cap : 64;
    L->blocks = (double*)realloc(L->blocks, sizeof(double) * 209 * L->cap);
    L->block_samples = (uint64_t*)realloc(L->block_samples, sizeof(uint64_t) * L->cap);
  }
  memcpy(L->blocks + 209 * L->nblocks, L->open, sizeof(L->open));
  L->block_samples[L->nblocks] = L->open_samples;
  L->nblocks += 1;
  memset(L->open, 0, sizeof(L->open));
  L->open_samples = 0;
}

static void sample(flbref3_lattice* L) {
  double f0[Q];
  for (int i = 0; i < Q; ++i)
    f0[i] = flbref3_equilibrium(i, L->p.rho0, L->p.ux0, L->p.uy0, L->p.uz0);
  for (size_t s = 0; s < L->N; ++s) {
    double d[Q];
    for (int i = 0; i < Q; ++i) d[i] = L->f[i * L->N + s] - f0[i];
    int q = 19;
    for (int i = 0; i < Q; ++i) L->open[i] += d[i];
    for (int i = 0; i < Q; ++i)
      for (int j = i; j < Q; ++j) L->open[q++] += d[i] * d[j];
  }
  L->open_samples += 1;
  if (L->p.block_steps > 0 && L->open_samples * (uint64_t)L->p.sample_every >=
                                  (uint64_t)L->p.block_steps)
    close_block(L);
}

int flbref3_lattice_step(flbref3_lattice* L, uint64_t nsteps) {
  const flbref3_params* p = &L->p;
  for (uint64_t n = 0; n < nsteps; ++n) {
    if (p->sample_every > 0 && L->t % (uint64_t)p->sample_every == 0) sample(L);
    for (int z = 0; z < p->nz; ++z)
      for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
          const size_t s = idx3(L, x, y, z);
          double f[Q], fo[Q];
          for (int i = 0; i < Q; ++i) f[i] = L->f[i * L->N + s];
          const int rc = flbref3_collide(p, f, s, L->t, fo);
          if (rc != FLBREF_OK) return rc;
          for (int i = 0; i < Q; ++i) {
            const int xd = (x + CX[i] + p->nx) % p->nx, yd = (y + CY[i] + p->ny) % p->ny;
            const int zd = (z + CZ[i] + p->nz) % p->nz;
            L->tmp[i * L->N + idx3(L, xd, yd, zd)] = fo[i];
          }
        }
    double* t = L->f;
    L->f = L->tmp;
    L->tmp = t;
    L->t += 1;
  }
  return FLBREF_OK;
}

int flbref3_lattice_read_populations(flbref3_lattice* L, double* f) {
  memcpy(f, L->f, sizeof(double) * Q * L->N);
  return FLBREF_OK;
}

static void cov_from(const double* sums, double n, double* mean, double* cov) {
  for (int i = 0; i < Q; ++i) mean[i] = sums[i] / n;
  int q = 19;
  for (int i = 0; i < Q; ++i)
    for (int j = i; j < Q; ++j) {
      const double c = sums[q++] / n - mean[i] * mean[j];
      cov[i * Q + j] = cov[j * Q + i] = c;
    }
}

int flbref3_lattice_read_covariance(flbref3_lattice* L, flbref3_cov* out) {
  memset(out, 0, sizeof(*out));
  double tot[209];
  memcpy(tot, L->open, sizeof(tot));
  uint64_t ns = L->open_samples;
  for (uint64_t b = 0; b < L->nblocks; ++b) {
    for (int v = 0; v < 209; ++v) tot[v] += L->blocks[209 * b + v];
    ns += L->block_samples[b];
  }
  out->nsamples = ns * L->N;
  out->nblocks = L->nblocks;
  if (ns == 0) return FLBREF_OK;
  cov_from(tot, (double)out->nsamples, out->mean_df, out->cov_f);
  if (L->nblocks >= 2) {
    double s1[361] = {0}, s2[361] = {0};
    for (uint64_t b = 0; b < L->nblocks; ++b) {
      double mean[Q], c[361];
      cov_from(L->blocks + 209 * b, (double)(L->block_samples[b] * L->N), mean, c);
      for (int k = 0; k < 361; ++k) {
        s1[k] += c[k];
        s2[k] += c[k] * c[k];
      }
    }
    const double nb = (double)L->nblocks;
    for (int k = 0; k < 361; ++k) {
      const double v = (s2[k] - s1[k] * s1[k] / nb) / (nb - 1.0);
      out->se_cov_f[k] = sqrt(v > 0 ? v / nb : 0.0);
    }
  }
  return FLBREF_OK;
}

int flbref3_lattice_reset_stats(flbref3_lattice* L) {
  memset(L->open, 0, sizeof(L->open));
  L->open_samples = 0;
  L->nblocks = 0;
  return FLBREF_OK;
}

uint64_t flbref3_lattice_time(flbref3_lattice* L) { return L->t; }

void flbref3_lattice_destroy(flbref3_lattice* L) {
  if (!L) return;
  free(L->f);
  free(L->tmp);
  free(L->blocks);
  free(L->block_samples);
  free(L);
}
