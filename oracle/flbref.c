/*
 * flbref.c — plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY; see flbref.h).
 *
 * Written for a reader who holds the paper: each function names the
 * section and equation it takes its steps from.  Nothing here is blocked,
 * fused or reordered beyond what those equations state.  Build with
 * -O2 -ffp-contract=off so that every product is rounded on its own.
 */
#include "flbref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* D2Q9 lattice (Fig. 1, App. A).  The velocity order is the column order
 * of the printed transform matrices (A3)/(A4): rest, the four axis
 * directions counter-clockwise from +x, then the four diagonals
 * counter-clockwise from (+1,+1). */
static const int VX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int VY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
/* Weights, eq. (A2). */
static const double W[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
/* Lattice temperature theta = c_s^2 = 1/3 (App. A, below eq. (A1)). */
static const double THETA = 1.0 / 3.0;

/* Forward Hermite-norm transform, eq. (A3): row a = moment
 * (rho, j_x, j_y, Pi_xx-yy, Pi_xy, Pi_xx+yy, q_x, q_y, eps), column i. */
static void hermite_matrix(double m[9][9]) {
  const double s3 = sqrt(3.0), s32 = sqrt(1.5), s6 = sqrt(6.0);
  const double t[9][9] = {
      {1, 1, 1, 1, 1, 1, 1, 1, 1},
      {0, s3, 0, -s3, 0, s3, -s3, -s3, s3},
      {0, 0, s3, 0, -s3, s3, s3, -s3, -s3},
      {0, 1.5, -1.5, 1.5, -1.5, 0, 0, 0, 0},
      {0, 0, 0, 0, 0, 3, -3, 3, -3},
      {-1, 0.5, 0.5, 0.5, 0.5, 2, 2, 2, 2},
      {0, -s32, 0, s32, 0, s6, -s6, -s6, s6},
      {0, 0, -s32, 0, s32, s6, s6, -s6, -s6},
      {0.5, -1, -1, -1, -1, 2, 2, 2, 2}};
  memcpy(m, t, sizeof(t));
}

void flbref_velocities(int32_t vx[9], int32_t vy[9], double w[9]) {
  for (int i = 0; i < 9; ++i) {
    vx[i] = VX[i];
    vy[i] = VY[i];
    w[i] = W[i];
  }
}

void flbref_hermite_matrix(double m[81]) {
  double t[9][9];
  hermite_matrix(t);
  memcpy(m, t, sizeof(t));
}

/* Second-order equilibrium, eq. (2) with theta = 1/3, i.e. eq. (A1). */
double flbref_equilibrium(int i, double rho, double ux, double uy) {
  const double uv = ux * VX[i] + uy * VY[i];
  const double uu = ux * ux + uy * uy;
  return rho * W[i] *
         (1.0 + uv / THETA + (uv * uv) / (2.0 * THETA * THETA) - uu / (2.0 * THETA));
}

/* ------------------------------------------------------------------ */
/* f-norm basis by classical Gram-Schmidt, Sec. IV.
 *
 * The scalar product is eq. (28) with the weight f_i^0 taken at unit
 * density, g_i = f_i^0(1, u): eq. (27) carries no rho, and with this
 * weight the density row stays the one-vector (text after eq. (32)).
 * The start vectors are the nine Hermite rows of eq. (A3) in table order;
 * the projection step is eq. (29) (classical: coefficients from the
 * original row m^a) and the normalisation of eq. (30) divides by the
 * square root of the squared norm, which is what eq. (27) requires.
 * Returns FLBREF_E_INVALID_VELOCITY when some g_i <= 0: the scalar product
 * is then not positive definite and the construction has no solution
 * (Fig. 11 and the text around it). */
static int gram_schmidt(const double g[9], double mt[9][9]) {
  double m[9][9];
  hermite_matrix(m);
  for (int i = 0; i < 9; ++i)
    if (!(g[i] > 0.0)) return FLBREF_E_INVALID_VELOCITY;
  for (int a = 0; a < 9; ++a) {
    double mhat[9];
    for (int i = 0; i < 9; ++i) mhat[i] = m[a][i];
    for (int b = 0; b < a; ++b) {
      double proj = 0.0; /* sum_j m~_j^b f_j^0 m_j^a */
      for (int j = 0; j < 9; ++j) proj += mt[b][j] * g[j] * m[a][j];
      for (int i = 0; i < 9; ++i) mhat[i] -= mt[b][i] * proj;
    }
    double nrm2 = 0.0;
    for (int j = 0; j < 9; ++j) nrm2 += mhat[j] * g[j] * mhat[j];
    if (!(nrm2 > 0.0)) return FLBREF_E_INVALID_VELOCITY;
    const double nrm = sqrt(nrm2);
    for (int i = 0; i < 9; ++i) mt[a][i] = mhat[i] / nrm;
  }
  return FLBREF_OK;
}

static void unit_weight(double ux, double uy, double g[9]) {
  for (int i = 0; i < 9; ++i) g[i] = flbref_equilibrium(i, 1.0, ux, uy);
}

int flbref_fnorm_basis(double ux, double uy, double mt[81]) {
  double g[9], t[9][9];
  unit_weight(ux, uy, g);
  const int rc = gram_schmidt(g, t);
  if (rc == FLBREF_OK) memcpy(mt, t, sizeof(t));
  return rc;
}

/* Look-up-table variant (Sec. IV, the paragraphs after Fig. 11): the basis
 * is taken at the nearest point of a 51 x 51 velocity grid with spacing
 * 0.02 covering [-0.5, 0.5]^2.  Nearest means floor(u/0.02 + 1/2).  A
 * velocity off the grid, or a grid point outside the validity region,
 * fails the same way the exact construction does. */
static const double LUT_DU = 0.02;
static const int LUT_HALF = 25;

static int lut_point(double ux, double uy, double ug[2]) {
  const double fx = floor(ux / LUT_DU + 0.5), fy = floor(uy / LUT_DU + 0.5);
  if (!(fabs(fx) <= LUT_HALF && fabs(fy) <= LUT_HALF)) return FLBREF_E_INVALID_VELOCITY;
  ug[0] = fx * LUT_DU;
  ug[1] = fy * LUT_DU;
  return FLBREF_OK;
}

int flbref_lut_basis(double ux, double uy, double mt[81], double ug[2]) {
  const int rc = lut_point(ux, uy, ug);
  if (rc != FLBREF_OK) return rc;
  return flbref_fnorm_basis(ug[0], ug[1], mt);
}

/* ------------------------------------------------------------------ */
/* Counter-based generator: Philox4x32 with 10 rounds (Salmon, Moraes,
 * Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11).
 * Round: two 32x32->64 products of counter words 0 and 2 with the two
 * Philox multipliers; the new words are (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1,
 * lo0); between rounds the key advances by the two Weyl constants. */
static const uint32_t PHILOX_M0 = 0xD2511F53u, PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u, PHILOX_W1 = 0xBB67AE85u;

void flbref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    const uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* The unit Gaussians N of eq. (6) for one site and one step.  The paper
 * only asks for independent unit-variance Gaussians; the draw used here:
 *   counter = (site lo, site hi, step lo, step hi XOR tag), key = seed;
 *   the 128 output bits give six 21-bit integers U_k,
 *     U_0..U_3 = top 21 bits of words 0..3,
 *     U_4 = (w0 & 0x7ff) | (w1 & 0x3ff) << 11,
 *     U_5 = (w2 & 0x7ff) | (w3 & 0x3ff) << 11,
 *   uniforms u_k = (U_k + 1/2) 2^-21 in (0, 1), and Box-Muller
 *   (Box & Muller 1958) on the pairs (u0,u1), (u2,u3), (u4,u5):
 *     r = sqrt(-2 ln u_even), N = (r cos 2 pi u_odd, r sin 2 pi u_odd). */
void flbref_site_gaussians(uint64_t seed, uint64_t site, uint64_t step, uint32_t tag,
                           double N[6]) {
  const uint32_t ctr[4] = {(uint32_t)site, (uint32_t)(site >> 32), (uint32_t)step,
                           (uint32_t)(step >> 32) ^ tag};
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4];
  flbref_philox4x32_10(ctr, key, w);
  uint32_t U[6];
  for (int k = 0; k < 4; ++k) U[k] = w[k] >> 11;
  U[4] = (w[0] & 0x7FFu) | ((w[1] & 0x3FFu) << 11);
  U[5] = (w[2] & 0x7FFu) | ((w[3] & 0x3FFu) << 11);
  const double two_pi = 2.0 * 3.14159265358979323846;
  for (int p = 0; p < 3; ++p) {
    const double ua = ((double)U[2 * p] + 0.5) / 2097152.0;
    const double ub = ((double)U[2 * p + 1] + 0.5) / 2097152.0;
    const double r = sqrt(-2.0 * log(ua));
    N[2 * p] = r * cos(two_pi * ub);
    N[2 * p + 1] = r * sin(two_pi * ub);
  }
}

/* Tag that separates the thermal-start draws from the step noise. */
static const uint32_t TAG_THERMAL = 0x80000000u;

/* ------------------------------------------------------------------ */
/* One collision at one site, Sec. II eq. (6) with the f-norm basis of
 * Sec. IV (or, for the Hermite variant, the fixed tables of App. A).
 *
 *   rho = sum f, u = sum f v / rho (text after eq. (1));
 *   M~^a = sum_i m~_i^a f_i (eq. (31)); M~^{a,0} = rho delta^{a0} (eq. (32));
 *   Lambda^{ab} = -delta^{ab} / tau^a (text before eq. (12));
 *   xi^a = sqrt(mu rho (2 tau^a - 1)) / tau^a (eq. (20) with the noise
 *     strength mu = kT / theta multiplying the variance; xi = 0 for the
 *     conserved rho, j_x, j_y);
 *   f*_i = f_i + sum_a n~_i^a [ -(M~^a - M~^{a,0}) / tau^a + xi^a N^a ]
 *     with n~_i^a = m~_i^a f_i^0(1,u) (the choice n = m f^0 / rho above
 *     eq. (18)).
 * For the conserved modes the bracket vanishes identically, so the sum
 * runs over a = 3..8. */
static int collide_with(const flbref_params* p, const double f[9], uint64_t site,
                        uint64_t step, const int32_t* grid_point, double fout[9]);

int flbref_collide(const flbref_params* p, const double f[9], uint64_t site, uint64_t step,
                   double fout[9]) {
  return collide_with(p, f, site, step, NULL, fout);
}

/* The table variant's collision with its basis taken at the grid point
 * u_g = (ix, iy) * 0.02 instead of the nearest one.  A local velocity that
 * lies exactly half-way between two grid points has two nearest points;
 * flbref_collide takes floor(u / 0.02 + 1/2), and this call gives the
 * collision at the other one, so that either reading can be checked. */
int flbref_collide_lut_at(const flbref_params* p, const double f[9], uint64_t site,
                          uint64_t step, int32_t ix, int32_t iy, double fout[9]) {
  if (p->basis != FLBREF_BASIS_FNORM_LUT) return FLBREF_E_ARG;
  if (ix < -LUT_HALF || ix > LUT_HALF || iy < -LUT_HALF || iy > LUT_HALF)
    return FLBREF_E_INVALID_VELOCITY;
  const int32_t g[2] = {ix, iy};
  return collide_with(p, f, site, step, g, fout);
}

static int collide_with(const flbref_params* p, const double f[9], uint64_t site,
                        uint64_t step, const int32_t* grid_point, double fout[9]) {
  double rho = 0.0, jx = 0.0, jy = 0.0;
  for (int i = 0; i < 9; ++i) {
    rho += f[i];
    jx += f[i] * VX[i];
    jy += f[i] * VY[i];
  }
  if (!(rho > 0.0) || !isfinite(jx) || !isfinite(jy)) return FLBREF_E_NONFINITE;
  const double ux = jx / rho, uy = jy / rho;

  double mt[9][9], nt[9][9], Meq[9];
  if (p->basis == FLBREF_BASIS_HERMITE) {
    /* App. A: m from (A3), n = w m (A4), equilibrium moments (A5). */
    hermite_matrix(mt);
    for (int a = 0; a < 9; ++a)
      for (int i = 0; i < 9; ++i) nt[a][i] = W[i] * mt[a][i];
    const double s3 = sqrt(3.0);
    Meq[0] = rho;
    Meq[1] = s3 * rho * ux;
    Meq[2] = s3 * rho * uy;
    Meq[3] = 1.5 * rho * (ux * ux - uy * uy);
    Meq[4] = 3.0 * rho * ux * uy;
    Meq[5] = 1.5 * rho * (ux * ux + uy * uy);
    Meq[6] = Meq[7] = Meq[8] = 0.0;
  } else if (p->basis == FLBREF_BASIS_FNORM_LUT) {
    double ug[2], g[9];
    int rc = FLBREF_OK;
    if (grid_point) {
      ug[0] = grid_point[0] * LUT_DU;
      ug[1] = grid_point[1] * LUT_DU;
    } else {
      rc = lut_point(ux, uy, ug);
    }
    if (rc != FLBREF_OK) return rc;
    unit_weight(ug[0], ug[1], g);
    rc = gram_schmidt(g, mt);
    if (rc != FLBREF_OK) return rc;
    for (int a = 0; a < 9; ++a)
      for (int i = 0; i < 9; ++i) nt[a][i] = mt[a][i] * g[i];
    /* Equilibrium moments projected onto the grid basis: the exact
     * sum_i m~_i^a(u_g) f_i^0(rho, u). */
    for (int a = 0; a < 9; ++a) {
      double s = 0.0;
      for (int i = 0; i < 9; ++i) s += mt[a][i] * flbref_equilibrium(i, rho, ux, uy);
      Meq[a] = s;
    }
  } else {
    double g[9];
    unit_weight(ux, uy, g);
    const int rc = gram_schmidt(g, mt);
    if (rc != FLBREF_OK) return rc;
    for (int a = 0; a < 9; ++a)
      for (int i = 0; i < 9; ++i) nt[a][i] = mt[a][i] * g[i];
    Meq[0] = rho;
    for (int a = 1; a < 9; ++a) Meq[a] = 0.0;
  }

  double M[9];
  for (int a = 0; a < 9; ++a) {
    double s = 0.0;
    for (int i = 0; i < 9; ++i) s += mt[a][i] * f[i];
    M[a] = s;
  }

  double N[6] = {0, 0, 0, 0, 0, 0};
  const double mu = p->kT / THETA;
  if (mu > 0.0) flbref_site_gaussians(p->seed, site, step, 0u, N);

  double dM[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int a = 3; a < 9; ++a) {
    const double tau = p->tau[a - 3];
    const double xi = sqrt(mu * rho * (2.0 * tau - 1.0)) / tau;
    dM[a] = -(M[a] - Meq[a]) / tau + xi * N[a - 3];
  }
  for (int i = 0; i < 9; ++i) {
    double s = 0.0;
    for (int a = 3; a < 9; ++a) s += nt[a][i] * dM[a];
    fout[i] = f[i] + s;
  }
  for (int i = 0; i < 9; ++i)
    if (!isfinite(fout[i])) return FLBREF_E_NONFINITE;
  return FLBREF_OK;
}

/* ------------------------------------------------------------------ */
/* Threads for the per-site loops of the lattice calls (1 unless set; the
 * results do not depend on it: every site and every Fourier coefficient is
 * computed on its own, and the correlator sums stay serial). */
static int g_threads = 1;

void flbref_set_threads(int n) { g_threads = n < 1 ? 1 : n; }

/* ------------------------------------------------------------------ */
/* Lattice: periodic nx x ny, populations f[i][y][x] (structure of arrays). */
#define MAX_TBLOCKS 1024

struct flbref_lattice {
  flbref_params p;
  size_t n;        /* sites */
  double* f;       /* 9 n */
  double* fpost;   /* 9 n, post-collision scratch */
  uint64_t t;
  int64_t err_step;
  /* measurement basis at (rho0, u0), Sec. IV (text after eq. (34)) */
  double mt0[9][9];
  double f00[9];
  /* correlator sums over (site, sample) */
  uint64_t ns;
  double S1[9], S2[81];
  /* time blocks for the standard error */
  uint64_t tb_len, tb_fill;
  double tb_S1[9], tb_S2[81];
  uint64_t nb;
  double (*blk_S1)[9];
  double (*blk_S2)[81];
  uint64_t* blk_n;
  /* structure-factor sums */
  uint64_t nsk;
  double* sk;      /* 5 n: |rho|^2, |jx|^2, |jy|^2, Re jx jy*, Im jx jy* */
  double* cosx; double* sinx; double* cosy; double* siny;
};

static int check_params(const flbref_params* p) {
  if (p->nx < 3 || p->ny < 3) return FLBREF_E_ARG;
  if (!(p->rho0 > 0.0) || !(p->kT >= 0.0)) return FLBREF_E_ARG;
  for (int a = 0; a < 6; ++a)
    if (!(p->tau[a] > 0.5)) return FLBREF_E_ARG;
  if (p->basis < 0 || p->basis > 2) return FLBREF_E_ARG;
  if (p->sample_every < 0 || p->sk_every < 0 || p->block_steps < 0) return FLBREF_E_ARG;
  double g[9];
  unit_weight(p->ux0, p->uy0, g);
  for (int i = 0; i < 9; ++i)
    if (!(g[i] > 0.0)) return FLBREF_E_INVALID_VELOCITY;
  return FLBREF_OK;
}

static void init_equilibrium(flbref_lattice* L) {
  const flbref_params* p = &L->p;
  for (int i = 0; i < 9; ++i) {
    const double v = flbref_equilibrium(i, p->rho0, p->ux0, p->uy0);
    for (size_t s = 0; s < L->n; ++s) L->f[i * L->n + s] = v;
  }
}

/* Ideal-gas start: f_i = f_i^0(rho0,u0) + sqrt(mu f_i^0) N_i, i.e. the
 * Poisson covariance of eq. (16) scaled by the noise strength.  The nine
 * Gaussians of a site come from two draws tagged apart from the step
 * noise (step field 0 -> N_0..N_5, step field 1 -> N_6..N_8). */
static void init_thermal(flbref_lattice* L) {
  const flbref_params* p = &L->p;
  const double mu = p->kT / THETA;
  for (size_t s = 0; s < L->n; ++s) {
    double Na[6], Nb[6], N9[9];
    flbref_site_gaussians(p->seed, s, 0, TAG_THERMAL, Na);
    flbref_site_gaussians(p->seed, s, 1, TAG_THERMAL, Nb);
    for (int k = 0; k < 6; ++k) N9[k] = Na[k];
    for (int k = 0; k < 3; ++k) N9[6 + k] = Nb[k];
    for (int i = 0; i < 9; ++i) {
      const double f0 = flbref_equilibrium(i, p->rho0, p->ux0, p->uy0);
      L->f[i * L->n + s] = f0 + sqrt(mu * f0) * N9[i];
    }
  }
}

int flbref_lattice_create(const flbref_params* p, flbref_lattice** out) {
  if (!p || !out) return FLBREF_E_ARG;
  const int rc = check_params(p);
  if (rc != FLBREF_OK) return rc;
  flbref_lattice* L = (flbref_lattice*)calloc(1, sizeof(*L));
  if (!L) return FLBREF_E_OOM;
  L->p = *p;
  L->n = (size_t)p->nx * (size_t)p->ny;
  L->f = (double*)malloc(9 * L->n * sizeof(double));
  L->fpost = (double*)malloc(9 * L->n * sizeof(double));
  L->sk = (double*)calloc(5 * L->n, sizeof(double));
  L->cosx = (double*)malloc((size_t)p->nx * sizeof(double));
  L->sinx = (double*)malloc((size_t)p->nx * sizeof(double));
  L->cosy = (double*)malloc((size_t)p->ny * sizeof(double));
  L->siny = (double*)malloc((size_t)p->ny * sizeof(double));
  L->blk_S1 = calloc(MAX_TBLOCKS, sizeof(*L->blk_S1));
  L->blk_S2 = calloc(MAX_TBLOCKS, sizeof(*L->blk_S2));
  L->blk_n = calloc(MAX_TBLOCKS, sizeof(uint64_t));
  if (!L->f || !L->fpost || !L->sk || !L->cosx || !L->sinx || !L->cosy || !L->siny ||
      !L->blk_S1 || !L->blk_S2 || !L->blk_n) {
    flbref_lattice_destroy(L);
    return FLBREF_E_OOM;
  }
  const double two_pi = 2.0 * 3.14159265358979323846;
  for (int k = 0; k < p->nx; ++k) {
    L->cosx[k] = cos(two_pi * k / p->nx);
    L->sinx[k] = sin(two_pi * k / p->nx);
  }
  for (int k = 0; k < p->ny; ++k) {
    L->cosy[k] = cos(two_pi * k / p->ny);
    L->siny[k] = sin(two_pi * k / p->ny);
  }
  double g0[9];
  unit_weight(p->ux0, p->uy0, g0);
  gram_schmidt(g0, L->mt0);
  for (int i = 0; i < 9; ++i) L->f00[i] = flbref_equilibrium(i, p->rho0, p->ux0, p->uy0);
  L->tb_len = p->block_steps > 0 ? (uint64_t)p->block_steps : 0;
  L->err_step = -1;
  if (p->init == FLBREF_INIT_THERMAL)
    init_thermal(L);
  else
    init_equilibrium(L);
  *out = L;
  return FLBREF_OK;
}

void flbref_lattice_destroy(flbref_lattice* L) {
  if (!L) return;
  free(L->f);
  free(L->fpost);
  free(L->sk);
  free(L->cosx);
  free(L->sinx);
  free(L->cosy);
  free(L->siny);
  free(L->blk_S1);
  free(L->blk_S2);
  free(L->blk_n);
  free(L);
}

int flbref_lattice_set_fields(flbref_lattice* L, const double* rho, const double* ux,
                              const double* uy) {
  for (size_t s = 0; s < L->n; ++s)
    for (int i = 0; i < 9; ++i) L->f[i * L->n + s] = flbref_equilibrium(i, rho[s], ux[s], uy[s]);
  return FLBREF_OK;
}

int flbref_lattice_set_populations(flbref_lattice* L, const double* f9xy, uint64_t t) {
  memcpy(L->f, f9xy, 9 * L->n * sizeof(double));
  L->t = t;
  return FLBREF_OK;
}

int flbref_lattice_read_populations(flbref_lattice* L, double* f9xy) {
  memcpy(f9xy, L->f, 9 * L->n * sizeof(double));
  return FLBREF_OK;
}

/* Moments of the current populations.  at = 0: f-norm at the local
 * velocity (eq. (31)); at = 1: f-norm at (rho0, u0), the measurement basis
 * of Sec. IV; at = 2: Hermite rows of eq. (A3). */
int flbref_lattice_read_moments(flbref_lattice* L, int32_t at, double* m9xy) {
  double mh[9][9];
  hermite_matrix(mh);
  for (size_t s = 0; s < L->n; ++s) {
    double f[9], mt[9][9];
    for (int i = 0; i < 9; ++i) f[i] = L->f[i * L->n + s];
    if (at == 0) {
      double rho = 0, jx = 0, jy = 0, g[9];
      for (int i = 0; i < 9; ++i) {
        rho += f[i];
        jx += f[i] * VX[i];
        jy += f[i] * VY[i];
      }
      unit_weight(jx / rho, jy / rho, g);
      if (gram_schmidt(g, mt) != FLBREF_OK) return FLBREF_E_INVALID_VELOCITY;
    } else if (at == 1) {
      memcpy(mt, L->mt0, sizeof(mt));
    } else if (at == 2) {
      memcpy(mt, mh, sizeof(mt));
    } else {
      return FLBREF_E_ARG;
    }
    for (int a = 0; a < 9; ++a) {
      double v = 0.0;
      for (int i = 0; i < 9; ++i) v += mt[a][i] * f[i];
      m9xy[a * L->n + s] = v;
    }
  }
  return FLBREF_OK;
}

/* Accumulate correlator sums of df = f - f^0(rho0,u0) over all sites
 * (eqs. (16), (23)) into the totals and into the open time block.  A
 * block closes after block_steps samples; when the block list is full,
 * neighbouring blocks merge pairwise and the block length doubles. */
static void sample_correlators(flbref_lattice* L) {
  double s1[9] = {0}, s2[81] = {0};
  for (size_t s = 0; s < L->n; ++s) {
    double df[9];
    for (int i = 0; i < 9; ++i) df[i] = L->f[i * L->n + s] - L->f00[i];
    for (int i = 0; i < 9; ++i) {
      s1[i] += df[i];
      for (int j = 0; j < 9; ++j) s2[i * 9 + j] += df[i] * df[j];
    }
  }
  for (int k = 0; k < 9; ++k) L->S1[k] += s1[k];
  for (int k = 0; k < 81; ++k) L->S2[k] += s2[k];
  L->ns += L->n;
  if (L->tb_len == 0) return;
  for (int k = 0; k < 9; ++k) L->tb_S1[k] += s1[k];
  for (int k = 0; k < 81; ++k) L->tb_S2[k] += s2[k];
  L->tb_fill += 1;
  if (L->tb_fill < L->tb_len) return;
  if (L->nb == MAX_TBLOCKS) {
    for (uint64_t b = 0; b < MAX_TBLOCKS / 2; ++b) {
      for (int k = 0; k < 9; ++k) L->blk_S1[b][k] = L->blk_S1[2 * b][k] + L->blk_S1[2 * b + 1][k];
      for (int k = 0; k < 81; ++k) L->blk_S2[b][k] = L->blk_S2[2 * b][k] + L->blk_S2[2 * b + 1][k];
      L->blk_n[b] = L->blk_n[2 * b] + L->blk_n[2 * b + 1];
    }
    L->nb = MAX_TBLOCKS / 2;
    L->tb_len *= 2;
  }
  memcpy(L->blk_S1[L->nb], L->tb_S1, sizeof(L->tb_S1));
  memcpy(L->blk_S2[L->nb], L->tb_S2, sizeof(L->tb_S2));
  L->blk_n[L->nb] = L->tb_fill * L->n;
  L->nb += 1;
  memset(L->tb_S1, 0, sizeof(L->tb_S1));
  memset(L->tb_S2, 0, sizeof(L->tb_S2));
  L->tb_fill = 0;
}

/* Field A of the structure factors at the current populations, measured
 * in the f-norm at (rho0, u0) (Sec. IV): which = 0 density, 1 and 2 the
 * momenta j~_x, j~_y (rows 1, 2 of m~(u0)); the reference value A_0 is
 * subtracted (text after eq. (26)). */
static double sk_field(const flbref_lattice* L, int which, size_t s) {
  double v = 0.0;
  if (which == 0) {
    for (int i = 0; i < 9; ++i) v += L->f[i * L->n + s];
    return v - L->p.rho0;
  }
  double ref = 0.0;
  for (int i = 0; i < 9; ++i) {
    v += L->mt0[which][i] * L->f[i * L->n + s];
    ref += L->mt0[which][i] * L->f00[i];
  }
  return v - ref;
}

/* Separable discrete Fourier transform dA(k) = sum_x dA(x) e^{-i k.x},
 * k = 2 pi (kx/nx, ky/ny), written out directly. */
static void dft2(const flbref_lattice* L, const double* a, double* re, double* im) {
  const int nx = L->p.nx, ny = L->p.ny;
  double* tr = (double*)malloc(L->n * sizeof(double));
  double* ti = (double*)malloc(L->n * sizeof(double));
#pragma omp parallel for schedule(static) num_threads(g_threads)
  for (int y = 0; y < ny; ++y)
    for (int kx = 0; kx < nx; ++kx) {
      double sr = 0.0, si = 0.0;
      for (int x = 0; x < nx; ++x) {
        const int ph = (int)(((long long)kx * x) % nx);
        sr += a[(size_t)y * nx + x] * L->cosx[ph];
        si -= a[(size_t)y * nx + x] * L->sinx[ph];
      }
      tr[(size_t)y * nx + kx] = sr;
      ti[(size_t)y * nx + kx] = si;
    }
#pragma omp parallel for schedule(static) num_threads(g_threads)
  for (int ky = 0; ky < ny; ++ky)
    for (int kx = 0; kx < nx; ++kx) {
      double sr = 0.0, si = 0.0;
      for (int y = 0; y < ny; ++y) {
        const int ph = (int)(((long long)ky * y) % ny);
        const double c = L->cosy[ph], sn = -L->siny[ph];
        const double ar = tr[(size_t)y * nx + kx], ai = ti[(size_t)y * nx + kx];
        sr += ar * c - ai * sn;
        si += ar * sn + ai * c;
      }
      re[(size_t)ky * nx + kx] = sr;
      im[(size_t)ky * nx + kx] = si;
    }
  free(tr);
  free(ti);
}

/* Accumulate |drho(k)|^2, |dj~_x(k)|^2, |dj~_y(k)|^2 and dj~_x(k) dj~_y(-k)
 * (eqs. (24)-(26); for real fields A(-k) is the conjugate of A(k)). */
static void sample_structure_factor(flbref_lattice* L) {
  const size_t n = L->n;
  double* a = (double*)malloc(n * sizeof(double));
  double* re = (double*)malloc(3 * n * sizeof(double));
  double* im = (double*)malloc(3 * n * sizeof(double));
  for (int w = 0; w < 3; ++w) {
    for (size_t s = 0; s < n; ++s) a[s] = sk_field(L, w, s);
    dft2(L, a, re + w * n, im + w * n);
  }
  for (size_t k = 0; k < n; ++k) {
    for (int w = 0; w < 3; ++w)
      L->sk[w * n + k] += re[w * n + k] * re[w * n + k] + im[w * n + k] * im[w * n + k];
    L->sk[3 * n + k] += re[n + k] * re[2 * n + k] + im[n + k] * im[2 * n + k];
    L->sk[4 * n + k] += im[n + k] * re[2 * n + k] - re[n + k] * im[2 * n + k];
  }
  L->nsk += 1;
  free(a);
  free(re);
  free(im);
}

/* One lattice update: optional sampling of the pre-collision state,
 * collision at every site, then streaming f_i(x + v_i, t+1) = f*_i(x, t)
 * with periodic wrap (eq. (1)). */
int flbref_lattice_step(flbref_lattice* L, uint64_t nsteps) {
  const int nx = L->p.nx, ny = L->p.ny;
  const size_t n = L->n;
  for (uint64_t k = 0; k < nsteps; ++k) {
    const uint64_t t = L->t;
    if (L->p.sample_every > 0 && t % (uint64_t)L->p.sample_every == 0) sample_correlators(L);
    if (L->p.sk_every > 0 && t % (uint64_t)L->p.sk_every == 0) sample_structure_factor(L);
    /* sites collide independently (rows spread over the threads); a failing
     * site leaves the populations unchanged and reports the lowest failing
     * site's error */
    size_t first_bad = n;
    int first_rc = FLBREF_OK;
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const size_t s = (size_t)y * nx + x;
        double f[9], fo[9];
        for (int i = 0; i < 9; ++i) f[i] = L->f[i * n + s];
        const int rc = flbref_collide(&L->p, f, s, t, fo);
        if (rc != FLBREF_OK) {
#pragma omp critical(flbref_bad_site)
          if (s < first_bad) {
            first_bad = s;
            first_rc = rc;
          }
        }
        for (int i = 0; i < 9; ++i) L->fpost[i * n + s] = fo[i];
      }
    if (first_bad < n) {
      L->err_step = (int64_t)t;
      return first_rc;
    }
    for (int i = 0; i < 9; ++i)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          const int xd = ((x + VX[i]) % nx + nx) % nx;
          const int yd = ((y + VY[i]) % ny + ny) % ny;
          L->f[i * n + (size_t)yd * nx + xd] = L->fpost[i * n + (size_t)y * nx + x];
        }
    L->t = t + 1;
  }
  return FLBREF_OK;
}

uint64_t flbref_lattice_time(flbref_lattice* L) { return L->t; }
int64_t flbref_lattice_error_step(flbref_lattice* L) { return L->err_step; }

int flbref_lattice_reset_stats(flbref_lattice* L) {
  L->ns = 0;
  memset(L->S1, 0, sizeof(L->S1));
  memset(L->S2, 0, sizeof(L->S2));
  memset(L->tb_S1, 0, sizeof(L->tb_S1));
  memset(L->tb_S2, 0, sizeof(L->tb_S2));
  L->tb_fill = 0;
  L->tb_len = L->p.block_steps > 0 ? (uint64_t)L->p.block_steps : 0;
  L->nb = 0;
  L->nsk = 0;
  memset(L->sk, 0, 5 * L->n * sizeof(double));
  return FLBREF_OK;
}

/* Covariance from raw sums: C = S2/n - (S1/n)(S1/n)^T. */
static void cov_from_sums(const double* S1, const double* S2, double n, double C[81]) {
  for (int i = 0; i < 9; ++i)
    for (int j = 0; j < 9; ++j) C[i * 9 + j] = S2[i * 9 + j] / n - (S1[i] / n) * (S1[j] / n);
}

/* Moment covariance B C B^T for a 9 x 9 row basis B (eq. (23)). */
static void transform_cov(const double B[9][9], const double C[81], double out[81]) {
  for (int a = 0; a < 9; ++a)
    for (int b = 0; b < 9; ++b) {
      double s = 0.0;
      for (int i = 0; i < 9; ++i)
        for (int j = 0; j < 9; ++j) s += B[a][i] * C[i * 9 + j] * B[b][j];
      out[a * 9 + b] = s;
    }
}

/* Correlators of the closed time blocks plus totals.  Standard errors are
 * the spread of the per-block estimates over sqrt(number of blocks). */
int flbref_lattice_read_covariance(flbref_lattice* L, flbref_cov* out) {
  memset(out, 0, sizeof(*out));
  double S1[9], S2[81];
  uint64_t ns = L->ns;
  for (int k = 0; k < 9; ++k) S1[k] = L->S1[k];
  for (int k = 0; k < 81; ++k) S2[k] = L->S2[k];
  out->nsamples = ns;
  out->nblocks = L->nb;
  if (ns == 0) return FLBREF_OK;
  for (int i = 0; i < 9; ++i) out->mean_df[i] = S1[i] / (double)ns;
  cov_from_sums(S1, S2, (double)ns, out->cov_f);
  transform_cov(L->mt0, out->cov_f, out->cov_m_fnorm_u0);
  double mh[9][9];
  hermite_matrix(mh);
  transform_cov(mh, out->cov_f, out->cov_m_hermite);
  if (L->nb >= 2) {
    double sf[81] = {0}, sf2[81] = {0}, sm[81] = {0}, sm2[81] = {0};
    for (uint64_t b = 0; b < L->nb; ++b) {
      double Cb[81], Mb[81];
      cov_from_sums(L->blk_S1[b], L->blk_S2[b], (double)L->blk_n[b], Cb);
      transform_cov(L->mt0, Cb, Mb);
      for (int k = 0; k < 81; ++k) {
        sf[k] += Cb[k];
        sf2[k] += Cb[k] * Cb[k];
        sm[k] += Mb[k];
        sm2[k] += Mb[k] * Mb[k];
      }
    }
    const double nb = (double)L->nb;
    for (int k = 0; k < 81; ++k) {
      const double vf = (sf2[k] - sf[k] * sf[k] / nb) / (nb - 1.0);
      const double vm = (sm2[k] - sm[k] * sm[k] / nb) / (nb - 1.0);
      out->se_cov_f[k] = sqrt(vf > 0 ? vf / nb : 0.0);
      out->se_cov_m[k] = sqrt(vm > 0 ? vm / nb : 0.0);
    }
  } else {
    for (int k = 0; k < 81; ++k) out->se_cov_f[k] = out->se_cov_m[k] = NAN;
  }
  return FLBREF_OK;
}

/* <|dA(k)|^2> / (nx ny) for which = 0..2, and the real (3) and imaginary
 * (4) parts of <dj~_x(k) dj~_y(-k)> / (nx ny); index ky*nx + kx. */
int flbref_lattice_read_structure_factor(flbref_lattice* L, int32_t which, double* out_xy) {
  if (which < 0 || which > 4) return FLBREF_E_ARG;
  const double norm = L->nsk > 0 ? 1.0 / ((double)L->nsk * (double)L->n) : 0.0;
  for (size_t k = 0; k < L->n; ++k) out_xy[k] = L->sk[which * L->n + k] * norm;
  return FLBREF_OK;
}

/* One Fourier coefficient sum_x dA(x) e^{-i k.x} of the current state. */
int flbref_lattice_read_fourier_mode(flbref_lattice* L, int32_t which, int32_t kx, int32_t ky,
                                     double out[2]) {
  if (which < 0 || which > 2) return FLBREF_E_ARG;
  const int nx = L->p.nx, ny = L->p.ny;
  double sr = 0.0, si = 0.0;
  const double two_pi = 2.0 * 3.14159265358979323846;
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      const double a = sk_field(L, which, (size_t)y * nx + x);
      const double ph = two_pi * ((double)(((long long)kx * x) % nx) / nx +
                                  (double)(((long long)ky * y) % ny) / ny);
      sr += a * cos(ph);
      si -= a * sin(ph);
    }
  out[0] = sr;
  out[1] = si;
  return FLBREF_OK;
}
