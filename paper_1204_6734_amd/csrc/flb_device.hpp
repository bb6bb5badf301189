// flb_device.hpp — per-site arithmetic of the fluctuating D2Q9 step on gfx950.
//
// Kaehler & Wagner, "A fluctuating lattice-Boltzmann method with improved
// Galilean invariance": the update of Sec. II, eq. (6), with the
// velocity-dependent f-norm moment basis of Sec. IV (eqs. (27)-(32)), the
// fixed Hermite basis of App. A, or the grid-velocity (table) variant of
// Sec. IV, plus the FDT noise amplitude of eq. (20).
//
// Design (not the paper's): the Gram-Schmidt of the nine Hermite rows
// under <a,b>_g = sum_i a_i g_i b_i, g = f^0(1,u), is carried out in closed
// form.  The three conserved rows are 1, sqrt3 (v_x - u_x), sqrt3 (v_y - u_y)
// exactly; the six others follow from the Cholesky factor L of the 6x6
// Schur complement G' = G - P P^T of the Hermite Gram matrix, whose entries
// are quadratic polynomials in u (G) and the projections P of the Hermite
// rows on the conserved rows (cubic).  Classical Gram-Schmidt with positive
// normalisation is exactly m~^{3..8} = L^-1 (m^{3..8} - projections), so
//   M~^{3..8} = L^-1 d,  d = Hermite non-equilibrium moments M - M^0(rho,u).
// The change df = sum_a m~^a g dM~^a has Hermite moments L dM~ (and no
// conserved ones), so df_i = w_i sum_a m_i^a (L dM~)_a; with one relaxation
// time for all six modes, L dM~ = L (xi N) - d / tau needs no solve at all.
// Nothing is tabulated and no 9x9 product is formed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "flb_kernels.hpp"
#include "fp64_series.hpp"

namespace flb {

// D2Q9 velocity set (Fig. 1; order of the columns of eqs. (A3)/(A4)).
constexpr int kVX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int kVY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int kOpp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

enum : int { kBasisFnormLocal = 0, kBasisHermite = 1, kBasisFnormLut = 2 };

// ------------------------------------------------------------------------
// Three-input XOR in one VALU instruction (gfx950 v_bitop3_b32 with truth
// table 0x96); the key operand is wave-uniform and stays in an SGPR.
__device__ __forceinline__ uint32_t xor3_vvs(uint32_t a, uint32_t b, uint32_t k) {
  uint32_t d;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(d) : "v"(a), "v"(b), "s"(k));
  return d;
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 products, word shuffle, key xor; key bumped by the Weyl
// increments between rounds.  Here the counter is (site, c1, c2, c3) with
// c1, c2, c3 and the key wave-uniform: the first round's product of word 2
// and the second round's product of word 0 are then wave-uniform too, and
// are written out so that they run on the scalar unit (18 per-lane products
// instead of 20).
__device__ __forceinline__ uint4 philox4x32_10_site(uint32_t site, uint32_t c1, uint32_t c2,
                                                   uint32_t c3, uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  // first Philox round, on (site, c1, c2, c3)
  uint64_t p0 = (uint64_t)M0 * (uint64_t)site;
  uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
  const uint32_t x1 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;        // uniform
  const uint32_t y1 = (uint32_t)p1;                          // uniform
  const uint32_t z1 = (uint32_t)(p0 >> 32) ^ (c3 ^ k1);      // per lane
  const uint32_t w1 = (uint32_t)p0;                          // per lane
  k0 += W0;
  k1 += W1;
  // second Philox round, on (x1, y1, z1, w1)
  p0 = (uint64_t)M0 * (uint64_t)x1;                          // uniform
  p1 = (uint64_t)M1 * (uint64_t)z1;
  uint4 c = make_uint4((uint32_t)(p1 >> 32) ^ (y1 ^ k0), (uint32_t)p1,
                       ((uint32_t)(p0 >> 32) ^ k1) ^ w1, (uint32_t)p0);
  k0 += W0;
  k1 += W1;
#pragma unroll
  for (int r = 2; r < 10; ++r) {
    p0 = (uint64_t)M0 * (uint64_t)c.x;
    p1 = (uint64_t)M1 * (uint64_t)c.z;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c = make_uint4(xor3_vvs(hi1, c.y, k0), lo1, xor3_vvs(hi0, c.w, k1), lo0);
    k0 += W0;
    k1 += W1;
  }
  return c;
}

// Two Gaussians of variance v from two BITS-bit integers ua, ub (Box-Muller
// on the uniforms (U + 1/2) 2^-BITS): r = sqrt(-2 v ln ua), angle 2 pi ub.
template <typename R, int BITS>
__device__ __forceinline__ void box_muller(uint32_t ua, uint32_t ub, R v, R& n0, R& n1);

// Hardware transcendentals: v_log_f32 is log2, v_sin/v_cos take the angle
// in revolutions, so r = sqrt(-2 v ln2 log2 ua) and the angle 2 pi ub needs
// no range reduction (ub in (0, 1)).  On the 2^21 inputs of the D2Q9 draw
// they agree with the correctly rounded values to ~1.3e-7 (absolute,
// sin/cos) and ~1.2e-7 (relative, log), the same level as the library
// routines.
// The pieces of one pair: the squared radius of unit variance l = -2 ln ua
// and the cosine and sine of the angle.
template <int BITS>
__device__ __forceinline__ void box_muller_parts_f32(uint32_t ua, uint32_t ub, float& l,
                                                     float& c, float& s) {
  constexpr float scale = 1.0f / (float)(1u << BITS), half = 0.5f / (float)(1u << BITS);
  const float fa = __fmaf_rn((float)ua, scale, half);
  const float fb = __fmaf_rn((float)ub, scale, half);
  l = -1.3862943611198906f * __builtin_amdgcn_logf(fa);
  c = __builtin_amdgcn_cosf(fb);
  s = __builtin_amdgcn_sinf(fb);
}
template <int BITS>
__device__ __forceinline__ void box_muller_f32(uint32_t ua, uint32_t ub, float v, float& n0,
                                               float& n1) {
  float l, c, s;
  box_muller_parts_f32<BITS>(ua, ub, l, c, s);
  const float r = __builtin_amdgcn_sqrtf(v * l);
  n0 = r * c;
  n1 = r * s;
}
template <>
__device__ __forceinline__ void box_muller<float, 21>(uint32_t ua, uint32_t ub, float v, float& n0,
                                                      float& n1) {
  box_muller_f32<21>(ua, ub, v, n0, n1);
}
template <>
__device__ __forceinline__ void box_muller<float, 24>(uint32_t ua, uint32_t ub, float v, float& n0,
                                                      float& n1) {
  box_muller_f32<24>(ua, ub, v, n0, n1);
}

// FP64 Box-Muller without library calls.  The inputs are integers, which
// makes exact argument reduction cheap:
// - ln x for x = (2 ua + 1) 2^-(B+1) in (0, 1): x = 2^e m with m in
//   [sqrt(1/2), sqrt(2)), ln m = 2 artanh z with z = (m - 1)/(m + 1),
//   |z| < 0.172, and ln x = e ln 2 + ln m;
// - the angle theta = 2 pi (ub + 1/2) 2^-B = pi K 2^-B with K = 2 ub + 1:
//   the octant is K >> (B - 2) and the rest an integer (taken from the
//   octant's far end in odd octants), so the reduced angle r = pi k 2^-B in
//   [0, pi/4] carries one rounding;
// - artanh, sin and cos on those intervals are the economised series of
//   fp64_series.hpp (truncation below 2^-57);
// - the radius sqrt(a) = a rsqrt(a) with the refined reciprocal square root.
// Each result is within a few ulp of the correctly rounded value.
template <int N>
__device__ __forceinline__ double horner(const double (&c)[N], double x) {
  double p = c[N - 1];
#pragma unroll
  for (int k = N - 2; k >= 0; --k) p = fma(p, x, c[k]);
  return p;
}
__device__ __forceinline__ double rsqrt_t(double x);
__device__ __forceinline__ double rcp_t(double x);

template <int BITS>
__device__ __forceinline__ double ln_uniform(uint32_t ua) {
  const double x = (double)(2u * ua + 1u) * (1.0 / (double)(2ull << BITS));  // exact
  const double mant = __builtin_amdgcn_frexp_mant(x);  // in [1/2, 1)
  const int ex = __builtin_amdgcn_frexp_exp(x);
  const bool low = mant < 0.70710678118654752440;
  const double m = low ? 2.0 * mant : mant;
  const int e = low ? ex - 1 : ex;
  const double z = (m - 1.0) * rcp_t(m + 1.0);
  const double p = horner(kAtanhSeries, z * z);
  return fma((double)e, 0.69314718055994530942, 2.0 * z * p);
}

template <int BITS>
__device__ __forceinline__ void sincos_uniform(uint32_t ub, double& sn, double& cs) {
  const uint32_t K = 2u * ub + 1u;
  const uint32_t oct = K >> (BITS - 2);
  const uint32_t rest = K & ((1u << (BITS - 2)) - 1u);
  const bool odd = (oct & 1u) != 0;
  const uint32_t k = odd ? (1u << (BITS - 2)) - rest : rest;
  const double r = (double)k * (3.14159265358979323846 / (double)(1u << BITS));
  const double r2 = r * r;
  const double ps = horner(kSinSeries, r2), pc = horner(kCosSeries, r2);
  // theta = Q pi/2 + a with a = r (even octant, Q = oct/2) or a = -r (odd
  // octant, Q = (oct + 1)/2 mod 4); (sin, cos)(Q pi/2 + a) =
  // (sin a, cos a), (cos a, -sin a), (-sin a, -cos a), (-cos a, sin a)
  const double sa = odd ? -(r * ps) : r * ps, ca = pc;
  const uint32_t Q = ((oct + 1u) >> 1) & 3u;
  const double s0 = (Q & 1u) ? ca : sa, c0 = (Q & 1u) ? sa : ca;
  sn = Q >= 2u ? -s0 : s0;
  cs = (Q == 1u || Q == 2u) ? -c0 : c0;
}

template <int BITS>
__device__ __forceinline__ void box_muller_f64(uint32_t ua, uint32_t ub, double v, double& n0,
                                               double& n1) {
  const double a = (-2.0 * v) * ln_uniform<BITS>(ua);
  const double r = a * rsqrt_t(a);
  double s, c;
  sincos_uniform<BITS>(ub, s, c);
  n0 = r * c;
  n1 = r * s;
}
template <>
__device__ __forceinline__ void box_muller<double, 21>(uint32_t ua, uint32_t ub, double v,
                                                       double& n0, double& n1) {
  box_muller_f64<21>(ua, ub, v, n0, n1);
}
template <>
__device__ __forceinline__ void box_muller<double, 24>(uint32_t ua, uint32_t ub, double v,
                                                       double& n0, double& n1) {
  box_muller_f64<24>(ua, ub, v, n0, n1);
}

// Six Gaussians of variance v for one (site, step, tag): the 128 Philox
// bits give six 21-bit integers (top 21 bits of each word, then the low 11
// bits of words 0/2 joined with the low 10 bits of words 1/3) for
// Box-Muller on the pairs (u0,u1), (u2,u3), (u4,u5).  v = 1 gives unit
// Gaussians (the collision's draw; it scales them by sqrt(rho), the
// local-density factor of the noise amplitude of eq. (20)).
// The six 21-bit integer pairs of one (site, step): counter (site, 0, step
// lo, step hi ^ tag) (a lattice has < 2^32 sites), the top 21 bits of each
// word and the low bits of words 0/2 joined with those of words 1/3.
struct Uniform21 {
  uint32_t a[3], b[3];
};
__device__ __forceinline__ Uniform21 site_uniforms(uint32_t k0, uint32_t k1, uint32_t site,
                                                   uint64_t step, uint32_t tag) {
  const uint4 w =
      philox4x32_10_site(site, 0u, (uint32_t)step, (uint32_t)(step >> 32) ^ tag, k0, k1);
  Uniform21 u;
  u.a[0] = w.x >> 11;
  u.b[0] = w.y >> 11;
  u.a[1] = w.z >> 11;
  u.b[1] = w.w >> 11;
  u.a[2] = (w.x & 0x7FFu) | ((w.y & 0x3FFu) << 11);
  u.b[2] = (w.z & 0x7FFu) | ((w.w & 0x3FFu) << 11);
  return u;
}

template <typename R>
__device__ __forceinline__ void site_gaussians(uint32_t k0, uint32_t k1, uint32_t site,
                                               uint64_t step, uint32_t tag, R v, R N[6]) {
  const Uniform21 u = site_uniforms(k0, k1, site, step, tag);
#pragma unroll
  for (int k = 0; k < 3; ++k) box_muller<R, 21>(u.a[k], u.b[k], v, N[2 * k], N[2 * k + 1]);
}

__device__ __forceinline__ float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }
// FP64 1/sqrt(x) and 1/x: the hardware estimates refined to within a few
// ulp of the correctly rounded values, at a fraction of the cost of sqrt and
// divide.  The gfx950 estimates r0 are good to 2^-24 relative (measured on
// 4M arguments over [2^-20, 2^20]).  With e the residual (e = 1 - x r0^2,
// resp. 1 - x r0), the exact values are r0 (1 - e)^(-1/2) = r0 (1 + e/2 +
// 3e^2/8 + ...) and r0 / (1 - e) = r0 (1 + e + e^2 + ...); one correction
// with the series to e^2 leaves a truncation of order e^3 ~ 2^-70, below
// the rounding of the few FP64 operations that form it (one step of the
// third-order method where two Newton steps took a few more operations).
// Arguments are positive and finite here (pivots and densities).
__device__ __forceinline__ double rsqrt_t(double x) {
  const double r = __builtin_amdgcn_rsq(x);
  const double e = fma(-(x * r), r, 1.0);
  return fma(r, e * fma(e, 0.375, 0.5), r);
}
__device__ __forceinline__ float rcp_t(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float sqrt_t(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrt_t(double x) { return sqrt(x); }
__device__ __forceinline__ double rcp_t(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r, 1.0);
  return fma(r, fma(e, e, e), r);
}

// Per-lattice constants of the collision, in the compute type.  The stored
// populations are h_i = f_i - f_i^0(rho0, u0): everything below works with
// differences from that reference state so that single precision keeps its
// relative accuracy on the small quantities (fluctuations, flow changes).
template <typename R>
struct CollideConst {
  R rho0, ux0, uy0;
  R rt[6];     // 1/tau^a, a = 3..8
  R xc[6];     // sqrt(mu (2 tau^a - 1)) / tau^a: xi^a = sqrt(rho) xc^a (eq. (20))
  R xc2;       // xc^2 when one_tau
  uint32_t k0, k1;
  int noise;   // 0 when kT == 0
  int one_tau; // the six relaxation times are equal
};

// Hermite moments (rows of eq. (A3)) of the shifted populations h; the
// moments of the reference f^0(rho0, u0) itself are rho0, rho0 u0 and the
// equilibrium values of eq. (A5).
template <typename R>
struct Moments {
  R drho, jx, jy;  // rho - rho0, j - rho0 u0
  R M3, M4, M5, M6, M7, M8;
};

template <typename R>
__device__ __forceinline__ Moments<R> hermite_moments(const R h[9]) {
  constexpr R S32 = R(1.2247448713915890491);  // sqrt(3/2)
  Moments<R> m;
  const R a13 = h[1] + h[3], a24 = h[2] + h[4];
  const R d13 = h[1] - h[3], d24 = h[2] - h[4];
  const R p57 = h[5] + h[7], p68 = h[6] + h[8];
  const R m57 = h[5] - h[7], m68 = h[6] - h[8];
  const R s58 = p57 + p68;
  const R dx = m57 - m68;   // h5 - h6 - h7 + h8
  const R dy = m57 + m68;   // h5 + h6 - h7 - h8
  const R dxy = p57 - p68;  // h5 - h6 + h7 - h8
  const R axis = a13 + a24;
  m.drho = (h[0] + axis) + s58;
  m.jx = d13 + dx;
  m.jy = d24 + dy;
  m.M3 = R(1.5) * (a13 - a24);
  m.M4 = R(3) * dxy;
  m.M5 = (R(0.5) * axis - h[0]) + R(2) * s58;
  m.M6 = S32 * (R(2) * dx - d13);
  m.M7 = S32 * (R(2) * dy - d24);
  m.M8 = (R(0.5) * h[0] - axis) + R(2) * s58;
  return m;
}

// sigma_i = sum_{a=3..8} m_i^a Y_a for the Hermite rows of eq. (A3).
template <typename R>
__device__ __forceinline__ void hermite_back(const R Y[6], R s[9]) {
  // written so that each product sits in the expression that adds it (one
  // fused multiply-add per term)
  constexpr R S32 = R(1.2247448713915890491), S6 = R(2.4494897427831780982);
  const R base = R(0.5) * Y[2] - Y[5];
  const R bp = base + R(1.5) * Y[0], bm = base - R(1.5) * Y[0];
  s[0] = R(0.5) * Y[5] - Y[2];
  s[1] = bp - S32 * Y[3];
  s[3] = bp + S32 * Y[3];
  s[2] = bm - S32 * Y[4];
  s[4] = bm + S32 * Y[4];
  const R db = R(2) * (Y[2] + Y[5]);
  const R dp = db + R(3) * Y[1], dm = db - R(3) * Y[1];
  const R q = Y[3] + Y[4], r = Y[3] - Y[4];
  s[5] = dp + S6 * q;
  s[7] = dp - S6 * q;
  s[6] = dm - S6 * r;
  s[8] = dm + S6 * r;
}

// g_i = f_i^0(1, u) of eq. (A1).
template <typename R>
__device__ __forceinline__ void unit_equilibrium(R bx, R by, R g[9]) {
  const R xx = bx * bx, yy = by * by;
  const R base = R(1) - R(1.5) * (xx + yy);
  const R c5 = bx + by, c6 = by - bx;
  const R ax = base + R(4.5) * xx, ay = base + R(4.5) * yy;
  const R d5 = base + R(4.5) * c5 * c5, d6 = base + R(4.5) * c6 * c6;
  g[0] = R(4.0 / 9.0) * base;
  g[1] = R(1.0 / 9.0) * (ax + R(3) * bx);
  g[3] = R(1.0 / 9.0) * (ax - R(3) * bx);
  g[2] = R(1.0 / 9.0) * (ay + R(3) * by);
  g[4] = R(1.0 / 9.0) * (ay - R(3) * by);
  g[5] = R(1.0 / 36.0) * (d5 + R(3) * c5);
  g[7] = R(1.0 / 36.0) * (d5 - R(3) * c5);
  g[6] = R(1.0 / 36.0) * (d6 + R(3) * c6);
  g[8] = R(1.0 / 36.0) * (d6 - R(3) * c6);
}

// Whether every g_i = f_i^0(1, u) of eq. (A1) is positive.  The weights are
// positive, so each sign is that of the bracket; the pair of opposite
// velocities +-c shares the bracket's even part e and has the smaller value
// e - 3 |u.c| (the same number as min(e + 3 u.c, e - 3 u.c) in any rounding).
template <typename R>
__device__ __forceinline__ bool valid_velocity(R bx, R by) {
  const R xx = bx * bx, yy = by * by;
  const R base = R(1) - R(1.5) * (xx + yy);
  const R c5 = bx + by, c6 = by - bx;
  const R ax = (base + R(4.5) * xx) - R(3) * fabs(bx);
  const R ay = (base + R(4.5) * yy) - R(3) * fabs(by);
  const R d5 = (base + R(4.5) * c5 * c5) - R(3) * fabs(c5);
  const R d6 = (base + R(4.5) * c6 * c6) - R(3) * fabs(c6);
  return fmin(fmin(base, fmin(ax, ay)), fmin(d5, d6)) > R(0);
}

// Local f-norm factors at basis velocity (bx, by): the Cholesky factor L of
// the Schur complement G' of the Hermite rows 3..8 under <,>_g (the Gram
// matrix with the projections on the conserved rows 1, m~^1, m~^2 taken out;
// Gram-Schmidt of eq. (11) in that order is the same factorisation), as its
// inverse pivots r[6], its diagonal and its strict lower part.
template <typename R>
struct Basis {
  R r[6];
  R dg[6];  // diagonal of the factor, sqrt(pivot) = pivot r
  R L[15];  // L10 L20 L21 L30 L31 L32 L40 L41 L42 L43 L50 L51 L52 L53 L54
};

template <typename R>
__device__ __forceinline__ void fnorm_basis(R bx, R by, Basis<R>& B) {
  constexpr R S3 = R(1.7320508075688772935), S6 = R(2.4494897427831780982);
  constexpr R H6 = R(1.2247448713915890491);  // sqrt6 / 2
  constexpr R T2 = R(2.1213203435596425732);  // 3 / sqrt2
  const R xx = bx * bx, yy = by * by, xy = bx * by, uu = xx + yy, dd = xx - yy;
  // conserved-row projections <1, m^a>_g, <m~^1, m^a>_g, <m~^2, m^a>_g
  const R P03 = R(1.5) * dd, P04 = R(3) * xy, P05 = R(1.5) * uu;
  R p1[5], p2[5];  // rows 3..7 (row 8 has none)
  p1[0] = S3 * bx * (R(1) - P03);
  p1[1] = S3 * by * (R(1) - R(3) * xx);
  p1[2] = S3 * bx * (R(1) - P05);
  p1[3] = T2 * yy;
  p1[4] = R(2) * T2 * xy;
  p2[0] = -S3 * by * (R(1) + P03);
  p2[1] = S3 * bx * (R(1) - R(3) * yy);
  p2[2] = S3 * by * (R(1) - P05);
  p2[3] = R(2) * T2 * xy;
  p2[4] = T2 * xx;
  // Hermite Gram matrix under g minus the conserved projections (lower part).
  const R A00 = (R(1) + R(0.75) * uu) - (P03 * P03 + p1[0] * p1[0] + p2[0] * p2[0]);
  const R A10 = -(P04 * P03 + p1[1] * p1[0] + p2[1] * p2[0]);
  const R A11 = (R(1) + R(3) * uu) - (P04 * P04 + p1[1] * p1[1] + p2[1] * p2[1]);
  const R A20 = R(0.75) * dd - (P05 * P03 + p1[2] * p1[0] + p2[2] * p2[0]);
  const R A21 = R(6) * xy - (P05 * P04 + p1[2] * p1[1] + p2[2] * p2[1]);
  const R A22 = (R(1) + R(0.75) * uu) - (P05 * P05 + p1[2] * p1[2] + p2[2] * p2[2]);
  const R A30 = -H6 * bx - (p1[3] * p1[0] + p2[3] * p2[0]);
  const R A31 = S6 * by - (p1[3] * p1[1] + p2[3] * p2[1]);
  const R A32 = H6 * bx - (p1[3] * p1[2] + p2[3] * p2[2]);
  const R A33 = (R(1) + R(3) * xx + R(1.5) * yy) - (p1[3] * p1[3] + p2[3] * p2[3]);
  const R A40 = H6 * by - (p1[4] * p1[0] + p2[4] * p2[0]);
  const R A41 = S6 * bx - (p1[4] * p1[1] + p2[4] * p2[1]);
  const R A42 = H6 * by - (p1[4] * p1[2] + p2[4] * p2[2]);
  const R A43 = R(6) * xy - (p1[4] * p1[3] + p2[4] * p2[3]);
  const R A44 = (R(1) + R(1.5) * xx + R(3) * yy) - (p1[4] * p1[4] + p2[4] * p2[4]);
  const R A50 = R(-1.5) * dd, A51 = R(6) * xy, A52 = R(1.5) * uu;
  const R A53 = S6 * bx, A54 = S6 * by, A55 = R(1) + R(1.5) * uu;
  // Cholesky, columns in Gram-Schmidt order.
  R* L = B.L;
  const R q0 = A00;
  const R r0 = rsqrt_t(q0);
  L[0] = A10 * r0; L[1] = A20 * r0; L[3] = A30 * r0; L[6] = A40 * r0; L[10] = A50 * r0;
  const R q1 = A11 - L[0] * L[0];
  const R r1 = rsqrt_t(q1);
  L[2] = (A21 - L[1] * L[0]) * r1;
  L[4] = (A31 - L[3] * L[0]) * r1;
  L[7] = (A41 - L[6] * L[0]) * r1;
  L[11] = (A51 - L[10] * L[0]) * r1;
  const R q2 = A22 - L[1] * L[1] - L[2] * L[2];
  const R r2 = rsqrt_t(q2);
  L[5] = (A32 - L[3] * L[1] - L[4] * L[2]) * r2;
  L[8] = (A42 - L[6] * L[1] - L[7] * L[2]) * r2;
  L[12] = (A52 - L[10] * L[1] - L[11] * L[2]) * r2;
  const R q3 = A33 - L[3] * L[3] - L[4] * L[4] - L[5] * L[5];
  const R r3 = rsqrt_t(q3);
  L[9] = (A43 - L[6] * L[3] - L[7] * L[4] - L[8] * L[5]) * r3;
  L[13] = (A53 - L[10] * L[3] - L[11] * L[4] - L[12] * L[5]) * r3;
  const R q4 = A44 - L[6] * L[6] - L[7] * L[7] - L[8] * L[8] - L[9] * L[9];
  const R r4 = rsqrt_t(q4);
  L[14] = (A54 - L[10] * L[6] - L[11] * L[7] - L[12] * L[8] - L[13] * L[9]) * r4;
  const R q5 = A55 - L[10] * L[10] - L[11] * L[11] - L[12] * L[12] - L[13] * L[13] -
               L[14] * L[14];
  const R r5 = rsqrt_t(q5);
  B.r[0] = r0; B.r[1] = r1; B.r[2] = r2; B.r[3] = r3; B.r[4] = r4; B.r[5] = r5;
  B.dg[0] = q0 * r0; B.dg[1] = q1 * r1; B.dg[2] = q2 * r2;
  B.dg[3] = q3 * r3; B.dg[4] = q4 * r4; B.dg[5] = q5 * r5;
}

// Forward substitution x = L^-1 d.
template <typename R>
__device__ __forceinline__ void lower_solve(const Basis<R>& B, const R d[6], R x[6]) {
  const R* L = B.L;
  x[0] = d[0] * B.r[0];
  x[1] = (d[1] - L[0] * x[0]) * B.r[1];
  x[2] = (d[2] - L[1] * x[0] - L[2] * x[1]) * B.r[2];
  x[3] = (d[3] - L[3] * x[0] - L[4] * x[1] - L[5] * x[2]) * B.r[3];
  x[4] = (d[4] - L[6] * x[0] - L[7] * x[1] - L[8] * x[2] - L[9] * x[3]) * B.r[4];
  x[5] = (d[5] - L[10] * x[0] - L[11] * x[1] - L[12] * x[2] - L[13] * x[3] - L[14] * x[4]) *
         B.r[5];
}

// Product y = L v with the full factor (diagonal included).
template <typename R>
__device__ __forceinline__ void lower_mul(const Basis<R>& B, const R v[6], R y[6]) {
  const R* L = B.L;
  y[0] = B.dg[0] * v[0];
  y[1] = B.dg[1] * v[1] + L[0] * v[0];
  y[2] = B.dg[2] * v[2] + L[1] * v[0] + L[2] * v[1];
  y[3] = B.dg[3] * v[3] + L[3] * v[0] + L[4] * v[1] + L[5] * v[2];
  y[4] = B.dg[4] * v[4] + L[6] * v[0] + L[7] * v[1] + L[8] * v[2] + L[9] * v[3];
  y[5] = B.dg[5] * v[5] + L[10] * v[0] + L[11] * v[1] + L[12] * v[2] + L[13] * v[3] +
         L[14] * v[4];
}

// Local state of a site from its shifted populations: rho, u, u - u0 and the
// non-equilibrium Hermite moments d = M(f) - M^0(rho,u) = M(h) - [M^0(rho,u) -
// M^0(rho0,u0)], the bracket of eq. (A5) written in differences.
template <typename R>
struct LocalState {
  Moments<R> m;
  R rho, ux, uy, dux, duy, sx, sy;
  R d[6];
};

template <typename R>
__device__ __forceinline__ bool local_state(const R h[9], R rho0, R ux0, R uy0,
                                            LocalState<R>& L) {
  L.m = hermite_moments(h);
  const Moments<R>& m = L.m;
  L.rho = rho0 + m.drho;
  if (!(L.rho > R(0)) || !(m.jx == m.jx) || !(m.jy == m.jy)) return false;
  const R inv = rcp_t(L.rho);
  // rho (u - u0) = (j - rho0 u0) - (rho - rho0) u0: small quantities only
  L.dux = (m.jx - m.drho * ux0) * inv;
  L.duy = (m.jy - m.drho * uy0) * inv;
  L.ux = ux0 + L.dux;
  L.uy = uy0 + L.duy;
  L.sx = L.ux + ux0;
  L.sy = L.uy + uy0;
  const R ex = rho0 * (L.dux * L.sx), ey = rho0 * (L.duy * L.sy);
  L.d[0] = m.M3 - R(1.5) * (m.drho * (L.ux * L.ux - L.uy * L.uy) + (ex - ey));
  L.d[1] = m.M4 - R(3) * (m.drho * (L.ux * L.uy) + rho0 * (L.dux * L.uy + ux0 * L.duy));
  L.d[2] = m.M5 - R(1.5) * (m.drho * (L.ux * L.ux + L.uy * L.uy) + (ex + ey));
  L.d[3] = m.M6;
  L.d[4] = m.M7;
  L.d[5] = m.M8;
  return true;
}

// The Gaussian draw of one (site, step).  It needs only the site and the
// step, so the step kernel makes it before the populations of the site have
// arrived; the collision scales it by sqrt(rho), the local-density factor of
// the amplitudes of eq. (20).  The draw keeps the Box-Muller pieces (the
// squared radius of unit variance l = -2 ln u, the cosine and the sine) and
// the collision forms the radius as sqrt(rho l), which folds that factor
// into the square root Box-Muller takes anyway.  NOISE32 (an FP64 collision
// on FP32 storage above the FP32 basis speed) draws unit Gaussians in FP32
// instead: the stored result is rounded to FP32 anyway, and the FP32
// transform is a sixth of the FP64 one's cost.
template <typename R, bool NOISE32>
struct SiteDraw {
  R l[3];   // -2 ln u of each pair
  R cs[6];  // cosine, sine of each pair's angle
};
template <>
struct SiteDraw<double, true> {
  double n[6];  // unit Gaussians, drawn in FP32
};

// The pieces of one FP64 pair (as box_muller_f64 without the radius).
template <int BITS>
__device__ __forceinline__ void box_muller_parts_f64(uint32_t ua, uint32_t ub, double& l,
                                                     double& c, double& s) {
  l = -2.0 * ln_uniform<BITS>(ua);
  sincos_uniform<BITS>(ub, s, c);
}

template <typename R, bool NOISE32>
__device__ __forceinline__ void site_draw(const CollideConst<R>& C, uint32_t site, uint64_t t,
                                          SiteDraw<R, NOISE32>& D) {
  if constexpr (NOISE32) {
    float n32[6];
    site_gaussians<float>(C.k0, C.k1, site, t, 0u, 1.0f, n32);
#pragma unroll
    for (int a = 0; a < 6; ++a) D.n[a] = R(n32[a]);
  } else {
    const Uniform21 u = site_uniforms(C.k0, C.k1, site, t, 0u);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if constexpr (sizeof(R) == 4)
        box_muller_parts_f32<21>(u.a[k], u.b[k], D.l[k], D.cs[2 * k], D.cs[2 * k + 1]);
      else
        box_muller_parts_f64<21>(u.a[k], u.b[k], D.l[k], D.cs[2 * k], D.cs[2 * k + 1]);
    }
  }
}

// sqrt(rho) N: the Gaussians with the local-density factor of eq. (20).
template <typename R, bool NOISE32>
__device__ __forceinline__ void scaled_noise(const SiteDraw<R, NOISE32>& D, R rho, R N[6]) {
  if constexpr (NOISE32) {
    const R sr = rho * rsqrt_t(rho);
#pragma unroll
    for (int a = 0; a < 6; ++a) N[a] = D.n[a] * sr;
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const R a = rho * D.l[k];
      R r;
      if constexpr (sizeof(R) == 4)
        r = sqrt_t(a);
      else
        r = a * rsqrt_t(a);  // a > 0: rho > 0 and u < 1
      N[2 * k] = r * D.cs[2 * k];
      N[2 * k + 1] = r * D.cs[2 * k + 1];
    }
  }
}

// One collision, eq. (6), on shifted populations h (in place), with the
// site's Gaussian draw (read only when the lattice has noise).  Returns
// error bits; on error h is left unchanged.
template <typename R, int BASIS, bool NOISE32>
__device__ __forceinline__ int collide(R h[9], const CollideConst<R>& C,
                                       const SiteDraw<R, NOISE32>& draw) {
  LocalState<R> S;
  if (!local_state(h, C.rho0, C.ux0, C.uy0, S)) return kErrNonFinite;
  const R ux = S.ux, uy = S.uy;
  const R* d = S.d;

  // With one relaxation time the f-norm collision scales the Gaussians by
  // the common coefficient as well: xi N = sqrt(xc^2 rho) N.
  const bool one = BASIS != kBasisHermite && C.one_tau;
  R N[6];
  if (C.noise) {
    scaled_noise(draw, one ? C.xc2 * S.rho : S.rho, N);
  } else {
#pragma unroll
    for (int a = 0; a < 6; ++a) N[a] = R(0);
  }

  // Hermite moments Y of the change of the populations, rows 3..8 (its
  // conserved moments vanish).
  R Y[6];
  if (BASIS == kBasisHermite) {
    // App. A: n = w m, relaxation of M - M^0 with the same amplitudes.
#pragma unroll
    for (int a = 0; a < 6; ++a) Y[a] = C.xc[a] * N[a] - C.rt[a] * d[a];
  } else {
    R bx = ux, by = uy;
    if (BASIS == kBasisFnormLut) {
      // nearest point of the 51 x 51 grid, spacing 0.02, [-0.5, 0.5]^2
      const R fx = floor(ux / R(0.02) + R(0.5)), fy = floor(uy / R(0.02) + R(0.5));
      if (!(fabs(fx) <= R(25) && fabs(fy) <= R(25))) return kErrInvalidVelocity;
      bx = fx * R(0.02);
      by = fy * R(0.02);
    }
    if (!valid_velocity(bx, by)) return kErrInvalidVelocity;
    // The change is df = sum_a n~^a dM~^a with n~^a = m~^a g (eq. (6)), a
    // g-weighted combination of the rows projected off the conserved ones.
    // Its conserved Hermite moments therefore vanish, and rows 3..8 give
    // G' y = L dM~ (G' = L L^T the Schur complement, y = L^-T dM~ the
    // coefficients of the projected rows).
    Basis<R> B;
    fnorm_basis(bx, by, B);
    if (one) {
      // One relaxation time: L (M~ / tau) = d / tau, so only the noise needs
      // the factor, Y = L (xi N) - d / tau.
      R LN[6];
      lower_mul(B, N, LN);
#pragma unroll
      for (int a = 0; a < 6; ++a) Y[a] = LN[a] - C.rt[0] * d[a];
    } else {
      R Mt[6], D[6];
      lower_solve(B, d, Mt);  // non-equilibrium f-norm moments M~^{3..8}
#pragma unroll
      for (int a = 0; a < 6; ++a) D[a] = C.xc[a] * N[a] - C.rt[a] * Mt[a];
      lower_mul(B, D, Y);
    }
  }
  // The Hermite rows are orthonormal under the weights w, so the change is
  // df_i = w_i sum_a m_i^a Y_a.
  R s[9];
  hermite_back(Y, s);
  constexpr R w0 = R(4.0 / 9.0), w1 = R(1.0 / 9.0), w5 = R(1.0 / 36.0);
  h[0] += w0 * s[0];
#pragma unroll
  for (int i = 1; i < 5; ++i) h[i] += w1 * s[i];
#pragma unroll
  for (int i = 5; i < 9; ++i) h[i] += w5 * s[i];
  return 0;
}

}  // namespace flb
