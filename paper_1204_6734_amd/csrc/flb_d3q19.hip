// flb_d3q19.hip — the fluctuating f-norm step on a D3Q19 lattice (gfx950).
//
// The paper builds its method on D2Q9 and notes that it carries over to
// other velocity sets (Sec. V).  This is that generalisation: the same
// collision in moment space (Sec. II, eq. (6)) with the FDT amplitude of
// eq. (20), in the basis obtained by Gram-Schmidt of 19 polynomial rows
// under g = f^0(1, u) (Sec. IV, eqs. (27)-(32)); the tables are in
// d3q19_tables.hpp.  As in D2Q9 the conserved rows are 1 and sqrt3 (v - u)
// in closed form and the fifteen others follow from the Cholesky factor of
// the 15x15 Schur complement of the Gram matrix, whose entries are
// quadratic polynomials in u (table kG3); populations are stored shifted by
// f^0(rho0, u0), SoA [19][nz][ny][nx], updated in place with the two-phase
// (AA) pattern, one 64 x 4 tile of one z plane per 256-thread workgroup.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "d3q19_tables.hpp"
#include "flb_buffer.hpp"
#include "flb_d3q19.hpp"
#include "flb_device.hpp"
#include "flb_reduce.hpp"

namespace flb {
namespace d3q19 {

constexpr double kS3 = 1.7320508075688772935;

template <typename R>
struct Const3 {
  R rho0, u0[3];
  R rt[15], xc[15];  // 1/tau, xi / sqrt(rho)
  R xc2;             // xc^2 when one_tau
  int one_tau;       // the fifteen relaxation times are equal
};

template <typename R>
__device__ __forceinline__ Const3<R> const3(const Desc3& d);
template <>
__device__ __forceinline__ Const3<float> const3<float>(const Desc3& d) {
  Const3<float> c;
  c.rho0 = d.rho0f;
  for (int a = 0; a < 3; ++a) c.u0[a] = d.u0f[a];
  for (int a = 0; a < 15; ++a) {
    c.rt[a] = d.rtf[a];
    c.xc[a] = d.xcf[a];
  }
  c.xc2 = d.xc2f;
  c.one_tau = d.one_tau;
  return c;
}
template <>
__device__ __forceinline__ Const3<double> const3<double>(const Desc3& d) {
  Const3<double> c;
  c.rho0 = d.rho0;
  for (int a = 0; a < 3; ++a) c.u0[a] = d.u0[a];
  for (int a = 0; a < 15; ++a) {
    c.rt[a] = d.rt[a];
    c.xc[a] = d.xc[a];
  }
  c.xc2 = d.xc2;
  c.one_tau = d.one_tau;
  return c;
}

// Fifteen Gaussians of variance v for one site and step (the step kernel
// draws unit ones and scales them by the square root of the local density):
// four Philox4x32-10 blocks with counter (site, block, step lo, step hi),
// key = seed; the top 24 bits of the sixteen words give uniforms
// (U + 1/2) 2^-24, and Box-Muller on consecutive pairs.
template <typename R>
__device__ __forceinline__ void gaussians15(uint32_t k0, uint32_t k1, uint32_t site, uint64_t t,
                                            R v, R N[15]) {
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const uint4 w = philox4x32_10_site(site, (uint32_t)c, (uint32_t)t, (uint32_t)(t >> 32), k0, k1);
    const uint32_t U[4] = {w.x >> 8, w.y >> 8, w.z >> 8, w.w >> 8};
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const int k = 4 * c + 2 * p;
      R n0, n1;
      box_muller<R, 24>(U[2 * p], U[2 * p + 1], v, n0, n1);
      if (k < 15) N[k] = n0;
      if (k + 1 < 15) N[k + 1] = n1;
    }
  }
}

// Every basis row is even or odd in the velocity (the start polynomials
// are, and the Gram-Schmidt under the symmetric weights keeps it; the
// tables are generated exactly so), and opposite velocities are adjacent
// (2k - 1, 2k), so sums over the nineteen directions fold into sums over
// the rest velocity and nine pairs.
constexpr int row_parity(int b) {
  int par = 0;
  for (int k = 1; k < 19; k += 2) {
    if (kM3[b][k] == 0.0 && kM3[b][k + 1] == 0.0) continue;
    const int p = kM3[b][k] == kM3[b][k + 1] ? 1 : (kM3[b][k] == -kM3[b][k + 1] ? -1 : 2);
    if (p == 2 || (par != 0 && p != par)) return 2;
    par = p;
  }
  return par == 0 ? 1 : par;
}
constexpr bool rows_have_parity() {
  for (int b = 0; b < 19; ++b) {
    if (row_parity(b) == 2) return false;
    if (row_parity(b) == -1 && kM3[b][0] != 0.0) return false;
  }
  for (int k = 1; k < 19; k += 2)
    if (kOpp3[k] != k + 1) return false;
  return true;
}
static_assert(rows_have_parity(), "basis rows must be even or odd, opposite velocities adjacent");

// c_i . v for one of the lattice velocities (components -1, 0, 1).
template <typename R>
__device__ __forceinline__ R cdot(int i, const R v[3]) {
  R s = R(0);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (kC3[i][a] > 0) s += v[a];
    if (kC3[i][a] < 0) s -= v[a];
  }
  return s;
}

// M_b = sum_i m^b_i h_i for all nineteen rows.
template <typename R>
__device__ __forceinline__ void moments3(const R h[19], R M[19]) {
  R hs[9], hd[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    hs[k] = h[2 * k + 1] + h[2 * k + 2];
    hd[k] = h[2 * k + 1] - h[2 * k + 2];
  }
#pragma unroll
  for (int b = 0; b < 19; ++b) {
    R s = kM3[b][0] != 0.0 ? R(kM3[b][0]) * h[0] : R(0);
#pragma unroll
    for (int k = 0; k < 9; ++k)
      if (kM3[b][2 * k + 1] != 0.0)
        s = fma(R(kM3[b][2 * k + 1]), row_parity(b) > 0 ? hs[k] : hd[k], s);
    M[b] = s;
  }
}

// sigma_i = sum_{b = 4..18} m^b_i y_{b-4}: the even rows give the part
// shared by a velocity and its opposite, the odd rows the part that flips.
template <typename R>
__device__ __forceinline__ void back3(const R y[15], R sg[19]) {
  R s0 = R(0);
#pragma unroll
  for (int b = 4; b < 19; ++b)
    if (kM3[b][0] != 0.0) s0 = fma(R(kM3[b][0]), y[b - 4], s0);
  sg[0] = s0;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    R e = R(0), o = R(0);
#pragma unroll
    for (int b = 4; b < 19; ++b) {
      if (kM3[b][2 * k + 1] == 0.0) continue;
      if (row_parity(b) > 0)
        e = fma(R(kM3[b][2 * k + 1]), y[b - 4], e);
      else
        o = fma(R(kM3[b][2 * k + 1]), y[b - 4], o);
    }
    sg[2 * k + 1] = e + o;
    sg[2 * k + 2] = e - o;
  }
}

// sqrt(rho) N from the site's unit Gaussians Nu (zeros without noise): the
// local-density factor of the amplitudes of eq. (20).
template <typename R>
__device__ __forceinline__ void scaled_noise(int noise, R rho, const R Nu[15], R N[15]) {
  if (noise) {
    const R sr = rho * rsqrt_t(rho);
#pragma unroll
    for (int a = 0; a < 15; ++a) N[a] = Nu[a] * sr;
  } else {
#pragma unroll
    for (int a = 0; a < 15; ++a) N[a] = R(0);
  }
}

// The collision in the fixed Hermite-type rows with n = w m (BASIS 1), on
// shifted populations h in place; returns error bits (h unchanged on error).
template <typename R, bool DRAW>
__device__ __forceinline__ int collide3_hermite(R h[19], const Const3<R>& C, int noise,
                                                const R Nu[15], uint32_t k0, uint32_t k1,
                                                uint32_t site, uint64_t t) {
  // moments of h in the basis rows (h = f - f^0(rho0, u0))
  R M[19];
  moments3(h, M);
  const R drho = M[0];
  const R rho = C.rho0 + drho;
  const R rs3 = R(1.0 / kS3);
  R du[3], u[3], su[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    // rho (u - u0) = (j - rho0 u0) - (rho - rho0) u0, with j - rho0 u0 = M^a / sqrt3
    du[a] = (M[1 + a] * rs3 - drho * C.u0[a]) * rcp_t(rho);
    u[a] = C.u0[a] + du[a];
    su[a] = u[a] + C.u0[a];
  }
  if (!(rho > R(0)) || !(du[0] == du[0]) || !(du[1] == du[1]) || !(du[2] == du[2]))
    return kErrNonFinite;
  // monomials of u (and their changes from u0, from small quantities)
  const R mono[9] = {u[0], u[1], u[2], u[0] * u[0], u[1] * u[1], u[2] * u[2],
                     u[0] * u[1], u[0] * u[2], u[1] * u[2]};
  const R dmono[9] = {du[0], du[1], du[2], du[0] * su[0], du[1] * su[1], du[2] * su[2],
                      du[0] * u[1] + C.u0[0] * du[1], du[0] * u[2] + C.u0[0] * du[2],
                      du[1] * u[2] + C.u0[1] * du[2]};
  // non-equilibrium moments d_b = M_b(f) - M_b(f^0(rho, u)), b = 4..18:
  // M_b(f^0(rho,u)) - M_b(f^0(rho0,u0)) = drho pi_b(u) + rho0 (pi_b(u) - pi_b(u0))
  R d[15];
#pragma unroll
  for (int b = 4; b < 19; ++b) {
    R pi = R(0), dpi = R(0);
#pragma unroll
    for (int k = 0; k < 9; ++k)
      if (kPi3[b][k] != 0.0) {
        pi += R(kPi3[b][k]) * mono[k];
        dpi += R(kPi3[b][k]) * dmono[k];
      }
    d[b - 4] = M[b] - (drho * pi + C.rho0 * dpi);
  }
  R N[15];
  if constexpr (DRAW) {
    // drawn here, with the local density folded into the Box-Muller radius
#pragma unroll
    for (int a = 0; a < 15; ++a) N[a] = R(0);
    if (noise) gaussians15<R>(k0, k1, site, t, rho, N);
  } else {
    scaled_noise(noise, rho, Nu, N);
  }

  // Hermite-type rows with n = w m: relax d directly
  R Y[15];
#pragma unroll
  for (int a = 0; a < 15; ++a) Y[a] = C.xc[a] * N[a] - C.rt[a] * d[a];
  R sg[19];
  back3(Y, sg);
#pragma unroll
  for (int i = 0; i < 19; ++i) h[i] += R(kW3[i]) * sg[i];
  return 0;
}

constexpr int kBlock3 = 256;   // threads per workgroup (one 64 x 4 tile)
// The factor L of the Schur complement G' = <m^a, m^b>_g - P0 P0^T -
// sum_a P_a P_a^T, one column at a time (packed lower part L[i(i+1)/2 + k]),
// and Y = L dM~ accumulated alongside: column j gives the pivot q and its
// inverse square root r, the column of L, and the contribution L_ij dM~_j
// to Y_i for i >= j (L_jj = q r); each row of the factor is dropped when its
// column is done.  dM~_j = -M~_j / tau_j + xi_j N_j needs the forward solve
// M~ = L^-1 d in column form (M~_j = d_j r, then d_i -= L_ij M~_j for i > j).
// With one relaxation time (ONE, N carrying xi) there is no solve:
// L (M~ / tau) = d / tau, so Y = L (xi N) - d / tau.
template <typename R, bool ONE>
__device__ __forceinline__ void factor_relax(const R mono[9], R uu, const R P0[15],
                                             const R P[3][15], R d[15], const R N[15],
                                             const Const3<R>& C, R Y[15]) {
  R L[120];
  if constexpr (ONE) {
    // -d / tau first, so that d is not held through the sweep
#pragma unroll
    for (int i = 0; i < 15; ++i) Y[i] = -(C.rt[0] * d[i]);
  }
#pragma unroll
  for (int j = 0; j < 15; ++j) {
#pragma unroll
    for (int i = j; i < 15; ++i) {
      R G = i == j ? R(1) - R(1.5) * uu : R(0);
#pragma unroll
      for (int k = 0; k < 9; ++k)
        if (kG3[4 + i][4 + j][k] != 0.0) G += R(kG3[4 + i][4 + j][k]) * mono[k];
      G = fma(-P0[i], P0[j], G);
#pragma unroll
      for (int c = 0; c < 3; ++c) G = fma(-P[c][i], P[c][j], G);
#pragma unroll
      for (int k = 0; k < j; ++k) G -= L[i * (i + 1) / 2 + k] * L[j * (j + 1) / 2 + k];
      L[i * (i + 1) / 2 + j] = G;
    }
    const R q = L[j * (j + 1) / 2 + j];
    const R r = rsqrt_t(q);
    R D;
    if constexpr (ONE) {
#pragma unroll
      for (int i = j + 1; i < 15; ++i) L[i * (i + 1) / 2 + j] *= r;
      D = N[j];
    } else {
      const R mj = d[j] * r;
#pragma unroll
      for (int i = j + 1; i < 15; ++i) {
        L[i * (i + 1) / 2 + j] *= r;
        d[i] -= L[i * (i + 1) / 2 + j] * mj;
      }
      D = C.xc[j] * N[j] - C.rt[j] * mj;
    }
    Y[j] = j == 0 && !ONE ? (q * r) * D : Y[j] + (q * r) * D;
#pragma unroll
    for (int i = j + 1; i < 15; ++i)
      Y[i] = j == 0 && !ONE ? L[i * (i + 1) / 2 + j] * D : Y[i] + L[i * (i + 1) / 2 + j] * D;
  }
}

// The f-norm collision (BASIS 0).  The change of the populations is
// df = sum_{a >= 4} n~^a dM~^a with n~^a = m~^a g and dM~^a = -M~^a / tau^a +
// xi^a N^a (eqs. (6), (20)): a g-weighted combination of the rows 4..18
// projected off the conserved ones 1, sqrt3 (v_a - u_a).  Its conserved
// moments vanish, and its moments on rows 4..18 are G' y = L dM~ (G' = L L^T
// the Schur complement of the Gram matrix, y = L^-T dM~ the coefficients of
// the projected rows).  The rows are orthonormal under the weights w, so
// df_i = w_i sum_b m^b_i (L dM~)_b, the back-transform of the Hermite-type
// collision.  L dM~ is accumulated column by column inside the Cholesky
// sweep (factor_relax).  Returns error bits; hout
// is written only on success (on failure the caller reads the site's values
// again).
template <typename R, bool ONE>
__device__ __forceinline__ int collide3_fnorm(const R h[19], const Const3<R>& C, int noise,
                                              const R Nu[15], R hout[19]) {
  R M[19];
  moments3(h, M);
  const R drho = M[0];
  const R rho = C.rho0 + drho;
  const R rs3 = R(1.0 / kS3);
  R du[3], u[3], su[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    du[a] = (M[1 + a] * rs3 - drho * C.u0[a]) * rcp_t(rho);
    u[a] = C.u0[a] + du[a];
    su[a] = u[a] + C.u0[a];
  }
  const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  // g of a velocity pair (c, -c) is w (t +- 3 c.u); the smaller is w (t - |3 c.u|)
  const R base = R(1) - R(1.5) * uu;
  R gmin = base;
#pragma unroll
  for (int k = 1; k < 19; k += 2) {
    const R cu = cdot<R>(k, u);
    gmin = fmin(gmin, (base + R(4.5) * cu * cu) - fabs(R(3) * cu));
  }
  if (!(rho > R(0)) || !(du[0] == du[0]) || !(du[1] == du[1]) || !(du[2] == du[2]))
    return kErrNonFinite;
  if (!(gmin > R(0))) return kErrInvalidVelocity;

  // with one relaxation time the Gaussians carry the common coefficient too:
  // xi N = sqrt(xc^2 rho) N
  R N[15];
  scaled_noise(noise, ONE ? C.xc2 * rho : rho, Nu, N);

  const R mono[9] = {u[0], u[1], u[2], u[0] * u[0], u[1] * u[1], u[2] * u[2],
                     u[0] * u[1], u[0] * u[2], u[1] * u[2]};
  const R dmono[9] = {du[0], du[1], du[2], du[0] * su[0], du[1] * su[1], du[2] * su[2],
                      du[0] * u[1] + C.u0[0] * du[1], du[0] * u[2] + C.u0[0] * du[2],
                      du[1] * u[2] + C.u0[1] * du[2]};
  // non-equilibrium moments d_b = M_b(f) - M_b(f^0(rho, u)), b = 4..18, and
  // the projections of rows 4..18 on the conserved rows 1, sqrt3 (v_a - u_a)
  R d[15], P0[15], P[3][15];
#pragma unroll
  for (int b = 4; b < 19; ++b) {
    R pi = R(0), dpi = R(0);
#pragma unroll
    for (int k = 0; k < 9; ++k)
      if (kPi3[b][k] != 0.0) {
        pi += R(kPi3[b][k]) * mono[k];
        dpi += R(kPi3[b][k]) * dmono[k];
      }
    d[b - 4] = M[b] - (drho * pi + C.rho0 * dpi);
    P0[b - 4] = pi;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      R ga = R(0);
#pragma unroll
      for (int k = 0; k < 9; ++k)
        if (kG3[1 + a][b][k] != 0.0) ga += R(kG3[1 + a][b][k]) * mono[k];
      P[a][b - 4] = ga - R(kS3) * u[a] * pi;
    }
  }
  R Y[15];
  factor_relax<R, ONE>(mono, uu, P0, P, d, N, C, Y);
  R sg[19];
  back3(Y, sg);
#pragma unroll
  for (int i = 0; i < 19; ++i) hout[i] = h[i] + R(kW3[i]) * sg[i];
  return 0;
}

// --------------------------------------------------------------- kernels
// Correlator statistics: q < 19 is the sum of df_q; the products df_i df_j,
// i <= j, follow row by row.
typedef double double4_v3 __attribute__((ext_vector_type(4)));

// Index of the product statistic (i, j), i <= j, in the layout above.
__device__ __forceinline__ int stat_pair(int i, int j) {
  return 19 + 19 * i - (i * (i - 1)) / 2 + (j - i);
}

// Correlator sums of df = h (the 209 statistics), added to this
// tile's partials; the whole workgroup calls this.  For one wavefront they
// are the entries of X^T X, X the 64 x 20 matrix of the nineteen df_i and a
// constant 1 per site, split into column blocks X0 (df_0..df_15) and X1
// (df_16..df_18, the constant, zeros): X0^T X0, X0^T X1 and X1^T X1 take
// sixteen FP64 matrix instructions each (16 x 16 output, four sites per
// instruction), on values the wavefront stages in LDS; lane l reads column
// l % 16 of site l / 16 of each group of four and holds output row
// l / 16 + 4 r, column l % 16 in element r.  The four wavefronts then add
// their sums in a fixed order.
template <typename S, typename R>
__device__ __forceinline__ void sample3(const R h[19], bool active, double* partials) {
  __shared__ S xs[4][64 * 19];
  __shared__ double red[4][224];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // the tile's open partial, read early so that its latency overlaps the sums
  const bool adds = threadIdx.x < kNStat3;
  const double open = adds ? partials[threadIdx.x] : 0.0;
  S* x = xs[wave];
#pragma unroll
  for (int i = 0; i < 19; ++i) x[lane * 19 + i] = active ? (S)h[i] : S(0);
  // the values come back from other lanes of the same wavefront, whose LDS
  // accesses complete in program order
  __builtin_amdgcn_wave_barrier();
  const int col = lane & 15, grp = lane >> 4;
  const int c1 = col < 3 ? 16 + col : 18;  // in-range column of block 1
  const double pad1 = col == 3 ? 1.0 : 0.0;
  double4_v3 a00 = {0.0, 0.0, 0.0, 0.0}, a01 = a00, a11 = a00;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const S* row = x + (4 * q + grp) * 19;
    const double v0 = (double)row[col];
    const S r1 = row[c1];
    const double v1 = col < 3 ? (double)r1 : pad1;
    a00 = __builtin_amdgcn_mfma_f64_16x16x4f64(v0, v0, a00, 0, 0, 0);
    a01 = __builtin_amdgcn_mfma_f64_16x16x4f64(v0, v1, a01, 0, 0, 0);
    a11 = __builtin_amdgcn_mfma_f64_16x16x4f64(v1, v1, a11, 0, 0, 0);
  }
  double* rw = red[wave];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = grp + 4 * r;  // output row, 0..15
    if (i <= col) rw[stat_pair(i, col)] = a00[r];
    if (col < 3) rw[stat_pair(i, 16 + col)] = a01[r];
    if (col == 3) rw[i] = a01[r];  // sum of df_i
  }
  if (grp < 3) {  // rows 16..18 of block 1 (element 0 of lanes 0..47)
    if (col < 3 && grp <= col) rw[stat_pair(16 + grp, 16 + col)] = a11[0];
    if (col == 3) rw[16 + grp] = a11[0];
  }
  __syncthreads();
  if (adds)
    partials[threadIdx.x] = open + ((red[0][threadIdx.x] + red[1][threadIdx.x]) +
                                    (red[2][threadIdx.x] + red[3][threadIdx.x]));
}

__device__ __forceinline__ uint32_t cell(int x, int y, int z, const Desc3& d) {
  return ((uint32_t)z * d.ny + y) * d.nx + x;
}

__device__ __forceinline__ int wrap(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// Wavefronts per SIMD the register allocation of a step variant aims at:
// three in FP32 (the one-relaxation-time f-norm collision fits in 163
// registers; the general one spills 32-40 bytes per lane there and still
// runs 1.5 % faster than at two), one in FP64.
template <typename R>
constexpr int waves3() {
  return sizeof(R) == 8 ? 1 : 3;
}

// One 64 x 4 tile of one z plane per workgroup, one wavefront per tile row,
// so y and z are wave-uniform: a site reads (and writes back) plane i at
// itself in the even phase, plane opp(i) at x - c_i in the odd phase.  The
// per-lane part of an offset is one of three columns x - 1, x, x + 1; the
// row part (nine distinct (y, z) shifts) is scalar.  Tiles are renumbered
// so that each XCD sweeps a contiguous range of z planes.
template <typename S, typename R, int BASIS, bool SAMPLE, int ODD, bool ONE>
__global__ __launch_bounds__(kBlock3) __attribute__((amdgpu_waves_per_eu(waves3<R>()))) void
step3_kernel(const Desc3* __restrict__ desc, const uint64_t* __restrict__ clock,
             uint32_t step_idx) {
  const Desc3& d = *desc;
  const uint64_t t = *clock + step_idx;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int z = tile / d.tiles_xy;
  const int rr = tile - z * d.tiles_xy;
  const int ty = rr / d.tiles_x, tx = rr - ty * d.tiles_x;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int x = tx * 64 + (threadIdx.x & 63), y = ty * 4 + wave;
  const bool active = x < d.nx && y < d.ny;
  const uint32_t N = (uint32_t)d.nx * d.ny * d.nz;
  constexpr uint32_t E = sizeof(S);
  // offsets of the site clamped onto the lattice: the lanes and wavefronts
  // of a ragged last tile load a real site's values (which they never use),
  // so the loads need no branch
  const int xl = x < d.nx ? x : d.nx - 1, yl = y < d.ny ? y : d.ny - 1;
  const uint32_t xc = (uint32_t)xl * E;
  uint32_t xm = xc - E, xp = xc + E;
  if (ODD && (tx == 0 || tx == d.tiles_x - 1)) {
    // wave-uniform: only the wavefronts at the two ends of a row wrap
    asm volatile("" : "+v"(xm), "+v"(xp));
    xm = xl == 0 ? (uint32_t)(d.nx - 1) * E : xm;
    xp = xl == d.nx - 1 ? 0u : xp;
  }
  uint32_t voff[19], soff[19];
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const int cx = ODD ? kC3[i][0] : 0, cy = ODD ? kC3[i][1] : 0, cz = ODD ? kC3[i][2] : 0;
    voff[i] = cx > 0 ? xm : (cx < 0 ? xp : xc);
    const int ys = cy == 0 ? yl : wrap(yl - cy, d.ny), zs = cz == 0 ? z : wrap(z - cz, d.nz);
    soff[i] = ((uint32_t)zs * d.ny + (uint32_t)ys) * (uint32_t)d.nx * E;
  }
  R h[19];
#pragma unroll
  for (int i = 0; i < 19; ++i)
    h[i] = (R)buf_load(plane_rsrc<S>(d.pop, N, ODD ? kOpp3[i] : i), voff[i], soff[i],
                       (S*)nullptr);
  // the unit Gaussians need only the site and the step: drawn here, while
  // the loads are still in flight, they cover part of the load latency
  // (measured faster for every variant but the FP32 Hermite-row one, which
  // is memory-bound and keeps drawing them inside its collision)
  constexpr bool kEarlyNoise = !(sizeof(R) == 4 && BASIS == 1);
  R Nu[15];  // read by the collision only where drawn
  if (kEarlyNoise && d.noise && active) gaussians15<R>(d.k0, d.k1, cell(x, y, z, d), t, R(1), Nu);
  if (SAMPLE) {
    if (d.sample_every > 0 && t % (uint64_t)d.sample_every == 0)
      sample3<S, R>(h, active, d.partials + (size_t)tile * kNStat3);
  }
  if (!active) return;
  const Const3<R> C = const3<R>(d);
  R hn[19];
  int e;
  if constexpr (BASIS == 0) {
    e = collide3_fnorm<R, ONE>(h, C, d.noise, Nu, hn);
  } else {
    e = collide3_hermite<R, !kEarlyNoise>(h, C, d.noise, Nu, d.k0, d.k1, cell(x, y, z, d), t);
#pragma unroll
    for (int i = 0; i < 19; ++i) hn[i] = h[i];
  }
  if (e) {
    // the lattice records the error and its step
    atomicOr(d.err, e);
    atomicMin(d.err_step, (unsigned long long)t);
  }
  // the plane resources are formed again for the stores from an opaque copy
  // of the base, so their SGPRs are not held through the collision
  void* pop_late = d.pop;
  asm volatile("" : "+s"(pop_late));
  if constexpr (BASIS == 0) {
    if (__builtin_amdgcn_ballot_w64(e != 0)) {
      // a site of this wavefront failed (rare): it streams uncollided, with
      // its values read again (nothing of this step is stored yet); the
      // branch is wave-uniform, so the buffer resources stay scalar
#pragma unroll
      for (int i = 0; i < 19; ++i) {
        const R v = (R)buf_load(plane_rsrc<S>(pop_late, N, ODD ? kOpp3[i] : i), voff[i], soff[i],
                                (S*)nullptr);
        hn[i] = e ? v : hn[i];
      }
    }
  }
  // the post-collision value of direction opp(i) goes back where i was read
#pragma unroll
  for (int i = 0; i < 19; ++i)
    buf_store(plane_rsrc<S>(pop_late, N, ODD ? kOpp3[i] : i), voff[i], soff[i], (S)hn[kOpp3[i]]);
}

// State I/O: f (unshifted FP64, [19][nz][ny][nx]) <-> storage at phase odd
// (odd: the reversed, un-streamed layout the next odd step reads).
template <typename S>
__global__ void io3_kernel(S* pop, double* f, Desc3 d, int odd, int to_storage) {
  const uint32_t N = (uint32_t)d.nx * d.ny * d.nz;
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= N) return;
  const int x = (int)(s % (uint32_t)d.nx);
  const int y = (int)((s / (uint32_t)d.nx) % (uint32_t)d.ny);
  const int z = (int)(s / ((uint32_t)d.nx * d.ny));
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    uint32_t e;
    if (!odd) {
      e = (uint32_t)i * N + s;
    } else {
      // f_i(x) is held in plane opp(i) at x - c_i
      const int xs = wrap(x - kC3[i][0], d.nx), ys = wrap(y - kC3[i][1], d.ny);
      const int zs = wrap(z - kC3[i][2], d.nz);
      e = (uint32_t)kOpp3[i] * N + ((uint32_t)zs * d.ny + ys) * d.nx + xs;
    }
    if (to_storage)
      pop[e] = (S)(f[(size_t)i * N + s] - d.shift[i]);
    else
      f[(size_t)i * N + s] = (double)pop[e] + d.shift[i];
  }
}

// Time blocks of the correlator sums (kNStat3 values per record); closing a
// block and the open sums: flb_reduce.hpp.
__global__ void merge_blocks3_kernel(double* rec, int nhalf) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= kNStat3) return;
  for (int b = 0; b < nhalf; ++b)
    rec[(size_t)b * kNStat3 + v] =
        rec[(size_t)(2 * b) * kNStat3 + v] + rec[(size_t)(2 * b + 1) * kNStat3 + v];
}

__global__ void fill3_kernel(double* p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// ------------------------------------------------------------- launchers
template <typename S, typename R, int BASIS, bool ONE>
static hipError_t step3_t(bool sample, int odd, int ntiles, const Desc3* d,
                          const uint64_t* clock, uint32_t k, hipStream_t st) {
  const dim3 g(ntiles), b(kBlock3);
  if (sample) {
    if (odd)
      hipLaunchKernelGGL((step3_kernel<S, R, BASIS, true, 1, ONE>), g, b, 0, st, d, clock, k);
    else
      hipLaunchKernelGGL((step3_kernel<S, R, BASIS, true, 0, ONE>), g, b, 0, st, d, clock, k);
  } else {
    if (odd)
      hipLaunchKernelGGL((step3_kernel<S, R, BASIS, false, 1, ONE>), g, b, 0, st, d, clock, k);
    else
      hipLaunchKernelGGL((step3_kernel<S, R, BASIS, false, 0, ONE>), g, b, 0, st, d, clock, k);
  }
  return hipGetLastError();
}

template <typename S>
static hipError_t step3_s(int basis, bool one_tau, bool sample, int odd, int ntiles,
                          const Desc3* d, const uint64_t* clock, uint32_t k, hipStream_t st) {
  if (basis == 1) return step3_t<S, S, 1, false>(sample, odd, ntiles, d, clock, k, st);
  if (one_tau) return step3_t<S, S, 0, true>(sample, odd, ntiles, d, clock, k, st);
  return step3_t<S, S, 0, false>(sample, odd, ntiles, d, clock, k, st);
}

hipError_t launch_step3(int storage, int basis, bool one_tau, bool sample, int odd, int ntiles,
                        const Desc3* d, const uint64_t* clock, uint32_t k, hipStream_t st) {
  if (storage == 0) return step3_s<double>(basis, one_tau, sample, odd, ntiles, d, clock, k, st);
  return step3_s<float>(basis, one_tau, sample, odd, ntiles, d, clock, k, st);
}

hipError_t launch_io3(int storage, void* pop, double* f, const Desc3& d, int odd, int to_storage,
                      hipStream_t st) {
  const uint32_t N = (uint32_t)d.nx * d.ny * d.nz;
  const dim3 g((N + 255) / 256), b(256);
  if (storage == 0)
    hipLaunchKernelGGL(io3_kernel<double>, g, b, 0, st, (double*)pop, f, d, odd, to_storage);
  else
    hipLaunchKernelGGL(io3_kernel<float>, g, b, 0, st, (float*)pop, f, d, odd, to_storage);
  return hipGetLastError();
}

hipError_t launch_close_block3(double* partials, int ntiles, double* record, hipStream_t st) {
  return close_block_sums<kNStat3>(partials, ntiles, record, st);
}
hipError_t launch_merge_blocks3(double* rec, int nhalf, hipStream_t st) {
  hipLaunchKernelGGL(merge_blocks3_kernel, dim3(1), dim3(256), 0, st, rec, nhalf);
  return hipGetLastError();
}
hipError_t launch_open_sum3(const double* partials, int ntiles, double* out, hipStream_t st) {
  return open_sums<kNStat3>(partials, ntiles, out, st);
}
hipError_t launch_fill3(double* p, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill3_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

}  // namespace d3q19
}  // namespace flb
