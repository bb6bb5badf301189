// flb_kernels.hip — utility kernels of libflb for gfx950 (MI355X): state
// input and output, moments, Fourier modes, time-block bookkeeping of the
// correlator sums, and the structure-factor transforms (eqs. (24)-(26)).
// The step kernel itself is in flb_step.hip.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "flb_device.hpp"
#include "flb_kernels.hpp"
#include "flb_reduce.hpp"

namespace flb {

// Element indices of the nine populations a site reads in phase `odd`, in
// the row-interleaved storage (value i of site (x, y) at (9 y + i) P + x,
// P the row pitch).  After the collision the value of direction kOpp[i]
// goes back to idx[i].
__device__ __forceinline__ void site_indices(int x, int y, int nx, int ny, int odd,
                                             uint32_t P, uint32_t idx[9]) {
  const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
  // start of plane row 0 of lattice rows y, y - 1, y + 1
  const uint32_t rc = 9u * y * P, rm = 9u * ym * P, rp = 9u * yp * P;
  if (!odd) {
#pragma unroll
    for (int i = 0; i < 9; ++i) idx[i] = rc + (uint32_t)i * P + x;
  } else {
    // plane opp(i) at x - v_i
    idx[0] = rc + x;
    idx[1] = rc + 3u * P + xm;   // v=( 1, 0): plane 3 at (x-1, y)
    idx[2] = rm + 4u * P + x;    // v=( 0, 1): plane 4 at (x, y-1)
    idx[3] = rc + 1u * P + xp;   // v=(-1, 0): plane 1 at (x+1, y)
    idx[4] = rp + 2u * P + x;    // v=( 0,-1): plane 2 at (x, y+1)
    idx[5] = rm + 7u * P + xm;   // v=( 1, 1): plane 7 at (x-1, y-1)
    idx[6] = rm + 8u * P + xp;   // v=(-1, 1): plane 8 at (x+1, y-1)
    idx[7] = rp + 5u * P + xp;   // v=(-1,-1): plane 5 at (x+1, y+1)
    idx[8] = rp + 6u * P + xm;   // v=( 1,-1): plane 6 at (x-1, y+1)
  }
}

// ---------------------------------------------------------------- state I/O
// Write f (unshifted FP64, natural order, [9][ny][nx]) into storage at phase
// `odd` (odd: the reversed, un-streamed layout the next odd step reads).
template <typename S>
__global__ void write_state_kernel(S* pop, uint32_t P, const double* __restrict__ f, int nx,
                                   int ny, int odd, Shift9 sh, int y0, int rows) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = y0 + (int)blockIdx.y;
  if (x >= nx) return;
  const uint32_t B = (uint32_t)nx * rows, bs = (uint32_t)blockIdx.y * nx + x;
  uint32_t idx[9];
  site_indices(x, y, nx, ny, odd, P, idx);
#pragma unroll
  for (int i = 0; i < 9; ++i) pop[idx[i]] = (S)(f[i * (size_t)B + bs] - sh.v[i]);
}

template <typename S>
__global__ void read_state_kernel(const S* __restrict__ pop, uint32_t P, double* f, int nx,
                                  int ny, int odd, Shift9 sh, int y0, int rows) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = y0 + (int)blockIdx.y;
  if (x >= nx) return;
  const uint32_t B = (uint32_t)nx * rows, bs = (uint32_t)blockIdx.y * nx + x;
  uint32_t idx[9];
  site_indices(x, y, nx, ny, odd, P, idx);
#pragma unroll
  for (int i = 0; i < 9; ++i) f[i * (size_t)B + bs] = (double)pop[idx[i]] + sh.v[i];
}

// Raw storage copy in natural (even-phase) order for checkpoints: keeps the
// stored bits exactly.
template <typename S>
__global__ void raw_state_kernel(S* pop, uint32_t P, S* buf, int nx, int ny, int odd, int to_buf,
                                 int y0, int rows) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = y0 + (int)blockIdx.y;
  if (x >= nx) return;
  const uint32_t B = (uint32_t)nx * rows, bs = (uint32_t)blockIdx.y * nx + x;
  uint32_t idx[9];
  site_indices(x, y, nx, ny, odd, P, idx);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    if (to_buf) buf[i * (size_t)B + bs] = pop[idx[i]];
    else pop[idx[i]] = buf[i * (size_t)B + bs];
  }
}

// Equilibrium f^0(rho(x), u(x)) from per-site fields (or uniform values when
// the field pointers are null), optionally plus ideal-gas fluctuations
// sqrt(mu f^0_i) N_i drawn with the thermal tag (two draws per site:
// step field 0 gives N_0..N_5, step field 1 gives N_6..N_8).
template <typename S>
__global__ void init_kernel(S* pop, uint32_t P, const double* __restrict__ rho,
                            const double* __restrict__ ux,
                            const double* __restrict__ uy, double rho0, double ux0, double uy0,
                            Shift9 sh, int nx, int ny, double mu, uint32_t k0, uint32_t k1,
                            int odd, int y0, int rows) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = y0 + (int)blockIdx.y;
  if (x >= nx) return;
  const uint32_t bs = (uint32_t)blockIdx.y * nx + x;  // index into band fields
  (void)rows;
  const uint32_t site = (uint32_t)y * nx + x;
  const double r = rho ? rho[bs] : rho0;
  const double vx = ux ? ux[bs] : ux0, vy = uy ? uy[bs] : uy0;
  double g[9];
  unit_equilibrium(vx, vy, g);
  double n9[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (mu > 0.0) {
    double a[6], b[6];
    site_gaussians<double>(k0, k1, site, 0, 0x80000000u, 1.0, a);
    site_gaussians<double>(k0, k1, site, 1, 0x80000000u, 1.0, b);
    for (int i = 0; i < 6; ++i) n9[i] = a[i];
    for (int i = 0; i < 3; ++i) n9[6 + i] = b[i];
  }
  uint32_t idx[9];
  site_indices(x, y, nx, ny, odd, P, idx);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const double f0 = r * g[i];
    const double f = mu > 0.0 ? f0 + sqrt(mu * f0) * n9[i] : f0;
    pop[idx[i]] = (S)(f - sh.v[i]);
  }
}

// Moments B f per site (B row-major 9x9 in global memory), or the local
// f-norm moments when B is null: M~^0 = rho, M~^1 = M~^2 = 0 (local
// velocity), M~^{3..8} = L^-1 d.
template <typename S>
__global__ void moments_kernel(const S* __restrict__ pop, uint32_t P,
                               const double* __restrict__ B, double* out, int nx, int ny, int odd,
                               double rho0, double ux0, double uy0, Shift9 sh, int* err, int y0,
                               int rows) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = y0 + (int)blockIdx.y;
  if (x >= nx) return;
  const uint32_t Bn = (uint32_t)nx * rows, bs = (uint32_t)blockIdx.y * nx + x;
  uint32_t idx[9];
  site_indices(x, y, nx, ny, odd, P, idx);
  double h[9], f[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    h[i] = (double)pop[idx[i]];
    f[i] = h[i] + sh.v[i];
  }
  if (B) {
    for (int a = 0; a < 9; ++a) {
      double sacc = 0.0;
      for (int i = 0; i < 9; ++i) sacc += B[a * 9 + i] * f[i];
      out[a * (size_t)Bn + bs] = sacc;
    }
    return;
  }
  LocalState<double> L;
  if (!local_state(h, rho0, ux0, uy0, L)) {
    atomicOr(err, kErrNonFinite);
    return;
  }
  double g[9];
  unit_equilibrium(L.ux, L.uy, g);
  double gmin = g[0];
  for (int i = 1; i < 9; ++i) gmin = fmin(gmin, g[i]);
  if (!(gmin > 0.0)) atomicOr(err, kErrInvalidVelocity);
  Basis<double> Bs;
  fnorm_basis(L.ux, L.uy, Bs);
  double Mt[6];
  lower_solve(Bs, L.d, Mt);
  out[bs] = L.rho;
  out[Bn + bs] = 0.0;
  out[2 * (size_t)Bn + bs] = 0.0;
  for (int a = 0; a < 6; ++a) out[(3 + a) * (size_t)Bn + bs] = Mt[a];
}

// Partial sums of one Fourier coefficient sum_x dA(x) e^{-i k.x} per block.
// A thread holds one column x at a time (256 consecutive columns per block,
// so the loads of a row are coalesced) and walks the rows y = blockIdx.y,
// blockIdx.y + gridDim.y, ...; e^{-i k.x} = e^{-2 pi i kx x / nx}
// e^{-2 pi i ky y / ny}, so the column's factor is evaluated once per column
// and the row's once per row (not at all for ky = 0).
template <typename S>
__global__ __launch_bounds__(256) void fourier_mode_kernel(const S* __restrict__ pop, uint32_t P,
                                                           double2* partial, int nx, int ny,
                                                           int odd, int which, int kx, int ky,
                                                           double ux0, double uy0) {
  __shared__ double sr[256], si[256];
  const int tid = threadIdx.x;
  double ar = 0.0, ai = 0.0;
  for (int x = blockIdx.x * 256 + tid; x < nx; x += gridDim.x * 256) {
    double cr = 0.0, ci = 0.0;  // sum over this thread's rows of dA e^{-i phi_y}
    for (int y = blockIdx.y; y < ny; y += gridDim.y) {
      uint32_t idx[9];
      site_indices(x, y, nx, ny, odd, P, idx);
      double h[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) h[i] = (double)pop[idx[i]];
      const Moments<double> m = hermite_moments(h);
      double a = m.drho;
      if (which == 1) a = 1.7320508075688772935 * (m.jx - ux0 * m.drho);
      if (which == 2) a = 1.7320508075688772935 * (m.jy - uy0 * m.drho);
      if (ky == 0) {
        cr += a;
      } else {
        const long long py = ((long long)ky * y) % ny;
        double sn, cs;
        sincospi(2.0 * ((double)py / ny), &sn, &cs);
        cr += a * cs;
        ci -= a * sn;
      }
    }
    const long long px = ((long long)kx * x) % nx;
    double sn, cs;
    sincospi(2.0 * ((double)px / nx), &sn, &cs);
    // (cr + i ci) (cs - i sn)
    ar += cr * cs + ci * sn;
    ai += ci * cs - cr * sn;
  }
  sr[tid] = ar;
  si[tid] = ai;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) {
      sr[tid] += sr[tid + o];
      si[tid] += si[tid + o];
    }
    __syncthreads();
  }
  if (tid == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = make_double2(sr[0], si[0]);
}

// ------------------------------------------------------------ time blocks
// Closing a block and the open sums: flb_reduce.hpp.

// Neighbouring records merge pairwise: rec[b] = rec[2b] + rec[2b+1].
__global__ void merge_blocks_kernel(double* rec, int nhalf) {
  const int v = threadIdx.x;
  if (v >= kNStat) return;
  for (int b = 0; b < nhalf; ++b)
    rec[(size_t)b * kNStat + v] = rec[(size_t)(2 * b) * kNStat + v] +
                                  rec[(size_t)(2 * b + 1) * kNStat + v];
}

__global__ void fill_kernel(double* p, size_t n, double value) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

// -------------------------------------------------------- structure factor
// The step kernel writes, on a structure-factor step, two complex planes
// z1 = d rho + i dj~_x and z2 = dj~_y (+ 0 i) of the lattice's storage
// precision T ([2][ny][nx]).  A 2-D FFT (rows, transpose, rows) follows, and
// the squared magnitudes are accumulated in FP64 over the half plane
// kx <= nx/2 (the other half follows from the fields being real).

template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return V{a.x + b.x, a.y + b.y}; }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return V{a.x - b.x, a.y - b.y}; }
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
  return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// multiplication by -i
template <typename V> __device__ __forceinline__ V cmi(V a) { return V{a.y, -a.x}; }

// In-register forward DFTs of 2, 4 and 8 points, out[r] = sum_s a[s]
// exp(-2 pi i r s / R), natural order in and out.
template <typename V> __device__ __forceinline__ void dft2(V* a) {
  const V t = a[1];
  a[1] = csub(a[0], t);
  a[0] = cadd(a[0], t);
}
template <typename V> __device__ __forceinline__ void dft4(V* a) {
  const V t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
  const V t2 = cadd(a[1], a[3]), t3 = cmi(csub(a[1], a[3]));
  a[0] = cadd(t0, t2);
  a[2] = csub(t0, t2);
  a[1] = cadd(t1, t3);
  a[3] = csub(t1, t3);
}
template <typename V> __device__ __forceinline__ void dft8(V* a) {
  using T = decltype(a[0].x);
  constexpr T h = T(0.70710678118654752440);
  V e[4] = {a[0], a[2], a[4], a[6]}, o[4] = {a[1], a[3], a[5], a[7]};
  dft4(e);
  dft4(o);
  // o[k] *= exp(-2 pi i k / 8)
  o[1] = V{h * (o[1].x + o[1].y), h * (o[1].y - o[1].x)};
  o[2] = cmi(o[2]);
  o[3] = V{h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y)};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    a[k] = cadd(e[k], o[k]);
    a[k + 4] = csub(e[k], o[k]);
  }
}
template <int R, typename V> __device__ __forceinline__ void dft(V* a) {
  if (R == 2) dft2(a);
  if (R == 4) dft4(a);
  if (R == 8) dft8(a);
}

// One Stockham pass of radix R over a row of length n held as E values per
// thread (thread t owns butterflies j = t + m n/E, m < E/R).  Ns is the
// length of the sub-transforms already done.  Input element j + r n/R of
// butterfly j is twiddled by w^(r k n/(Ns R)) (k = j mod Ns, w = e^{-2 pi
// i/n}) and transformed; output r goes to (j - k) R + k + r Ns.
template <int R, int E, typename V>
__device__ __forceinline__ void pass_load(V (&a)[E], const V* __restrict__ src, int n, int t) {
  const int tpr = n / E;
#pragma unroll
  for (int m = 0; m < E / R; ++m)
#pragma unroll
    for (int r = 0; r < R; ++r) a[m * R + r] = src[t + m * tpr + r * (n / R)];
}

// Twiddle w^k = exp(-2 pi i k / n), k < n, n a power of two.  FP64 reads the
// table; FP32 evaluates it with the hardware sine and cosine, which take the
// angle in revolutions (k / n is exact), to ~1e-7, the level of the FP32
// transform itself: the table's gathers from L2 stalled every pass (a row
// pass ran at half the speed it reaches without them).
__device__ __forceinline__ double2 twiddle(const double2* __restrict__ tw, int k, int) {
  return tw[k];
}
__device__ __forceinline__ float2 twiddle(const float2* __restrict__, int k, int n) {
  const float a = (float)k * (1.0f / (float)n);
  return float2{__builtin_amdgcn_cosf(a), -__builtin_amdgcn_sinf(a)};
}

// w^(r step) for the r-th input of a butterfly, w1 = w^step.  FP64 reads
// the table; FP32 takes products of w1 (w^2 = w1 w1, w^3 = w^2 w1, ...):
// one sine and cosine per butterfly instead of one per input, each power
// within a few FP32 roundings of the exact value.
template <typename V>
__device__ __forceinline__ V twiddle_pow(const V* __restrict__ tw, int step, int r, int n, V w1);
template <>
__device__ __forceinline__ double2 twiddle_pow<double2>(const double2* __restrict__ tw, int step,
                                                        int r, int, double2) {
  return tw[r * step];
}
template <>
__device__ __forceinline__ float2 twiddle_pow<float2>(const float2* __restrict__, int, int r, int,
                                                      float2 w1) {
  float2 w = w1;
  for (int q = 1; q < r; ++q) w = cmul(w, w1);
  return w;
}

template <int R, int E, typename V>
__device__ __forceinline__ void pass_compute(V (&a)[E], int n, int t, int Ns,
                                             const V* __restrict__ tw) {
  const int tpr = n / E;
#pragma unroll
  for (int m = 0; m < E / R; ++m) {
    if (Ns > 1) {
      const int j = t + m * tpr;
      const int step = (j & (Ns - 1)) * (n / (Ns * R));
      const V w1 = twiddle(tw, step, n);
#pragma unroll
      for (int r = 1; r < R; ++r) a[m * R + r] = cmul(a[m * R + r], twiddle_pow<V>(tw, step, r, n, w1));
    }
    dft<R>(&a[m * R]);
  }
}

template <int R, int E, typename V>
__device__ __forceinline__ void pass_store(const V (&a)[E], V* dst, int n, int t, int Ns) {
  const int tpr = n / E;
#pragma unroll
  for (int m = 0; m < E / R; ++m) {
    const int j = t + m * tpr;
    const int k = j & (Ns - 1);
    const int base = (j - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[base + r * Ns] = a[m * R + r];
  }
}

// Pass of run-time radix R: phase 0 loads (when src is given) and
// transforms, phase 1 stores.
template <int E, typename V>
__device__ __forceinline__ void fft_pass(int R, int phase, V (&a)[E], const V* src, V* dst,
                                         int n, int t, int Ns, const V* tw) {
  if (phase == 0) {
    if (R == 8) {
      if (src) pass_load<8, E>(a, src, n, t);
      pass_compute<8, E>(a, n, t, Ns, tw);
    } else if (R == 4) {
      if (src) pass_load<4, E>(a, src, n, t);
      pass_compute<4, E>(a, n, t, Ns, tw);
    } else {
      if (src) pass_load<2, E>(a, src, n, t);
      pass_compute<2, E>(a, n, t, Ns, tw);
    }
  } else {
    if (R == 8) pass_store<8, E>(a, dst, n, t, Ns);
    else if (R == 4) pass_store<4, E>(a, dst, n, t, Ns);
    else pass_store<2, E>(a, dst, n, t, Ns);
  }
}

// Forward FFT of `rows` rows of length n = 2^logn >= 8 (out-of-place, natural
// order), n / E threads per row and blockDim.x / (n / E) rows per workgroup,
// each row staged in LDS between passes.  Passes: one of radix 2 or 4 if
// logn is not a multiple of 3, then radix 8.  tw[m] = exp(-2 pi i m / n).
template <typename T, int E>
__global__ __launch_bounds__(1024) void fft_rows_kernel(const typename Cplx<T>::type* __restrict__ in,
                                                       typename Cplx<T>::type* out, int n, int logn,
                                                       int rows,
                                                       const typename Cplx<T>::type* __restrict__ tw) {
  using V = typename Cplx<T>::type;
  extern __shared__ unsigned char fft_lds[];
  const int tpr = n / E;
  const int lr = threadIdx.x / tpr, t = threadIdx.x - lr * tpr;
  const int rpb = blockDim.x / tpr;
  const size_t row = (size_t)blockIdx.x * rpb + lr;
  const bool have = row < (size_t)rows;
  V* buf = reinterpret_cast<V*>(fft_lds) + (size_t)lr * n;
  const V* src = in + (have ? row : 0) * n;
  V* dst = out + (have ? row : 0) * n;
  const int rem = logn % 3;
  const int npass = logn / 3 + (rem ? 1 : 0);
  V a[E];
  int Ns = 1;
  for (int p = 0; p < npass; ++p) {
    const int R = (p == 0 && rem) ? (1 << rem) : 8;
    if (p == 0) {
      // from global memory; a row past the end transforms zeros
      if (!have) {
#pragma unroll
        for (int e = 0; e < E; ++e) a[e] = V{T(0), T(0)};
      }
      fft_pass<E, V>(R, 0, a, have ? src : nullptr, nullptr, n, t, Ns, tw);
    } else {
      fft_pass<E, V>(R, 0, a, buf, nullptr, n, t, Ns, tw);
      __syncthreads();  // every read of this pass precedes its writes
    }
    if (p == npass - 1) {
      if (have) fft_pass<E, V>(R, 1, a, nullptr, dst, n, t, Ns, tw);
    } else {
      fft_pass<E, V>(R, 1, a, nullptr, buf, n, t, Ns, tw);
      __syncthreads();
    }
    Ns *= R;
  }
}
// Direct DFT of rows of any length n: out[k] = sum_j in[j] tw[(j k) mod n],
// tw[m] = exp(-2 pi i m / n), m < n; sums in FP64.
template <typename T>
__global__ void dft_rows_kernel(const typename Cplx<T>::type* __restrict__ in,
                                typename Cplx<T>::type* out, int n,
                                const typename Cplx<T>::type* __restrict__ tw) {
  using V = typename Cplx<T>::type;
  const size_t row = blockIdx.y;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const V* src = in + row * n;
  double sr = 0.0, si = 0.0;
  int m = 0;
  for (int j = 0; j < n; ++j) {
    const V a = src[j], wv = tw[m];
    sr += (double)a.x * wv.x - (double)a.y * wv.y;
    si += (double)a.x * wv.y + (double)a.y * wv.x;
    m += k;
    if (m >= n) m -= n;
  }
  out[row * n + k] = V{(T)sr, (T)si};
}

// out[c][r] = in[r][c] for gridDim.z matrices of rows x cols complex values,
// through 32 x 32 tiles in LDS (256 threads, 8 or 16 KB of LDS: more
// workgroups per CU than with 64 x 64 tiles).  The tiles are taken in
// diagonal order: block b of a matrix takes tile row b mod gy and tile column
// (b / gy + b mod gy) mod gx (a bijection of the gx x gy grid), so blocks
// that run together read and write segments of different rows and columns
// rather than all at one offset of the power-of-two row stride.
constexpr int kTransposeTile = 32;

template <typename V>
__global__ __launch_bounds__(256) void transpose_kernel(const V* __restrict__ in, V* out,
                                                        int rows, int cols) {
  constexpr int TILE = kTransposeTile, STEP = 256 / TILE;
  __shared__ V tile[TILE][TILE + 1];
  const int gx = gridDim.x, gy = gridDim.y;
  const int b = blockIdx.y * gx + blockIdx.x;
  const int tr = b % gy, tc = (b / gy + tr) % gx;
  const int bx = tc * TILE, by = tr * TILE;
  const size_t z = blockIdx.z;
  const V* src = in + z * (size_t)rows * cols;
  V* dst = out + z * (size_t)rows * cols;
  const int tx = threadIdx.x % TILE, ty = threadIdx.x / TILE;
#pragma unroll
  for (int q = 0; q < TILE / STEP; ++q) {
    const int j = ty + STEP * q, r = by + j, c = bx + tx;
    if (r < rows && c < cols) tile[j][tx] = src[(size_t)r * cols + c];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < TILE / STEP; ++q) {
    const int j = ty + STEP * q, c = bx + j, r = by + tx;
    if (r < rows && c < cols) dst[(size_t)c * rows + r] = tile[tx][j];
  }
}

// Accumulate |d rho(k)|^2, |dj~_x(k)|^2, |dj~_y(k)|^2 and dj~_x(k) dj~_y(-k)
// (real and imaginary part) over the half plane kx <= nx/2, from the
// transformed planes stored transposed ([kx][ky]).  With z1 = a + i b for
// real a, b: a(k) = (Z1(k) + conj Z1(-k))/2, b(k) = (Z1(k) - conj Z1(-k))/(2i);
// likewise c(k) = (Z2(k) + conj Z2(-k))/2 for the real z2.  Each value is
// thereby exactly the conjugate of its partner at -k.
template <typename T>
__global__ void sk_accumulate_kernel(const typename Cplx<T>::type* __restrict__ Zt, double* acc,
                                     int nx, int ny) {
  using V = typename Cplx<T>::type;
  const uint32_t N = (uint32_t)nx * ny;
  const uint32_t H = (uint32_t)(nx / 2 + 1) * ny;  // half-plane size
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= H) return;
  const int kx = (int)(i / (uint32_t)ny), ky = (int)(i - (uint32_t)kx * ny);
  const int mkx = kx == 0 ? 0 : nx - kx, mky = ky == 0 ? 0 : ny - ky;
  const uint32_t ip = (uint32_t)kx * ny + ky, im = (uint32_t)mkx * ny + mky;
  const V z = Zt[ip], zm = Zt[im], c0 = Zt[N + ip], cm = Zt[N + im];
  const double ar = 0.5 * ((double)z.x + zm.x), ai = 0.5 * ((double)z.y - zm.y);
  const double br = 0.5 * ((double)z.y + zm.y), bi = -0.5 * ((double)z.x - zm.x);
  const double cr = 0.5 * ((double)c0.x + cm.x), ci = 0.5 * ((double)c0.y - cm.y);
  acc[i] += ar * ar + ai * ai;
  acc[H + i] += br * br + bi * bi;
  acc[2u * H + i] += cr * cr + ci * ci;
  acc[3u * H + i] += br * cr + bi * ci;  // Re(b conj c)
  acc[4u * H + i] += bi * cr - br * ci;  // Im(b conj c)
}

static dim3 row_grid(int nx, int rows) { return dim3((nx + 255) / 256, rows); }

// The row-parallel utility kernels below process the band of rows
// [y0, y0 + rows); their host-side arrays hold that band only.
hipError_t launch_write_state(int storage, void* pop, uint32_t P, const double* f, int nx, int ny,
                              int odd, const Shift9& sh, int y0, int rows, hipStream_t st) {
  if (storage == 0)
    hipLaunchKernelGGL(write_state_kernel<double>, row_grid(nx, rows), dim3(256), 0, st,
                       (double*)pop, P, f, nx, ny, odd, sh, y0, rows);
  else
    hipLaunchKernelGGL(write_state_kernel<float>, row_grid(nx, rows), dim3(256), 0, st,
                       (float*)pop, P, f, nx, ny, odd, sh, y0, rows);
  return hipGetLastError();
}

hipError_t launch_read_state(int storage, const void* pop, uint32_t P, double* f, int nx, int ny,
                             int odd, const Shift9& sh, int y0, int rows, hipStream_t st) {
  if (storage == 0)
    hipLaunchKernelGGL(read_state_kernel<double>, row_grid(nx, rows), dim3(256), 0, st,
                       (const double*)pop, P, f, nx, ny, odd, sh, y0, rows);
  else
    hipLaunchKernelGGL(read_state_kernel<float>, row_grid(nx, rows), dim3(256), 0, st,
                       (const float*)pop, P, f, nx, ny, odd, sh, y0, rows);
  return hipGetLastError();
}

hipError_t launch_raw_state(int storage, void* pop, uint32_t P, void* buf, int nx, int ny, int odd,
                            int to_buf, int y0, int rows, hipStream_t st) {
  if (storage == 0)
    hipLaunchKernelGGL(raw_state_kernel<double>, row_grid(nx, rows), dim3(256), 0, st,
                       (double*)pop, P, (double*)buf, nx, ny, odd, to_buf, y0, rows);
  else
    hipLaunchKernelGGL(raw_state_kernel<float>, row_grid(nx, rows), dim3(256), 0, st,
                       (float*)pop, P, (float*)buf, nx, ny, odd, to_buf, y0, rows);
  return hipGetLastError();
}

hipError_t launch_init(int storage, void* pop, uint32_t P, const double* rho, const double* ux,
                       const double* uy, double rho0, double ux0, double uy0, const Shift9& sh,
                       int nx, int ny, double mu, uint32_t k0, uint32_t k1, int odd, int y0,
                       int rows, hipStream_t st) {
  if (storage == 0)
    hipLaunchKernelGGL(init_kernel<double>, row_grid(nx, rows), dim3(256), 0, st, (double*)pop,
                       P, rho, ux, uy, rho0, ux0, uy0, sh, nx, ny, mu, k0, k1, odd, y0, rows);
  else
    hipLaunchKernelGGL(init_kernel<float>, row_grid(nx, rows), dim3(256), 0, st, (float*)pop,
                       P, rho, ux, uy, rho0, ux0, uy0, sh, nx, ny, mu, k0, k1, odd, y0, rows);
  return hipGetLastError();
}

hipError_t launch_moments(int storage, const void* pop, uint32_t P, const double* B, double* out,
                          int nx,
                          int ny, int odd, double rho0, double ux0, double uy0,
                          const Shift9& sh, int* err, int y0, int rows, hipStream_t st) {
  if (storage == 0)
    hipLaunchKernelGGL(moments_kernel<double>, row_grid(nx, rows), dim3(256), 0, st,
                       (const double*)pop, P, B, out, nx, ny, odd, rho0, ux0, uy0, sh, err, y0,
                       rows);
  else
    hipLaunchKernelGGL(moments_kernel<float>, row_grid(nx, rows), dim3(256), 0, st,
                       (const float*)pop, P, B, out, nx, ny, odd, rho0, ux0, uy0, sh, err, y0,
                       rows);
  return hipGetLastError();
}

int fourier_mode_grid(int nx, int ny, int max_blocks, int* gx, int* gy) {
  const int cols = (nx + 255) / 256;
  *gx = cols < max_blocks ? cols : max_blocks;
  const int rows = max_blocks / *gx;
  *gy = rows < 1 ? 1 : (rows < ny ? rows : ny);
  return *gx * *gy;
}

hipError_t launch_fourier_mode(int storage, const void* pop, uint32_t P, double2* partial,
                               int max_blocks, int nx, int ny, int odd, int which, int kx, int ky,
                               double ux0, double uy0, hipStream_t st) {
  int gx, gy;
  fourier_mode_grid(nx, ny, max_blocks, &gx, &gy);
  const dim3 grid(gx, gy);
  if (storage == 0)
    hipLaunchKernelGGL(fourier_mode_kernel<double>, grid, dim3(256), 0, st, (const double*)pop, P,
                       partial, nx, ny, odd, which, kx, ky, ux0, uy0);
  else
    hipLaunchKernelGGL(fourier_mode_kernel<float>, grid, dim3(256), 0, st, (const float*)pop, P,
                       partial, nx, ny, odd, which, kx, ky, ux0, uy0);
  return hipGetLastError();
}

hipError_t launch_close_block(double* partials, int ntiles, double* record, hipStream_t st) {
  return close_block_sums<kNStat>(partials, ntiles, record, st);
}

hipError_t launch_close_block_many(double* const* partials, double* const* records,
                                  size_t record_offset, int n, int ntiles, hipStream_t st) {
  return close_block_sums_many<kNStat>(partials, records, record_offset, n, ntiles, st);
}

hipError_t launch_merge_blocks(double* rec, int nhalf, hipStream_t st) {
  hipLaunchKernelGGL(merge_blocks_kernel, dim3(1), dim3(64), 0, st, rec, nhalf);
  return hipGetLastError();
}

hipError_t launch_open_sum(const double* partials, int ntiles, double* out, hipStream_t st) {
  return open_sums<kNStat>(partials, ntiles, out, st);
}

hipError_t launch_fill(double* p, size_t n, double v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

// ------------------------------------------------- bandwidth probe
// A plain copy between two contiguous buffers, 16 bytes per lane: the
// device's streaming ceiling, independent of the populations' layout.
__global__ void stream_copy_kernel(const float4* __restrict__ in, float4* __restrict__ out,
                                   size_t n4) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n4) out[i] = in[i];
}

hipError_t launch_stream_copy(const void* in, void* out, size_t n4, hipStream_t st) {
  hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, st,
                     (const float4*)in, (float4*)out, n4);
  return hipGetLastError();
}

static bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }
static int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

// Values per thread of the LDS FFT for a row of length n, or 0 when rows of
// that length go through the direct DFT (not a power of two, shorter than
// 8, or longer than the LDS holds).
static int fft_values_per_thread(int n, size_t elem, size_t max_lds) {
  if (!is_pow2(n) || n < 8 || (size_t)n * elem > max_lds) return 0;
  return n <= 8192 ? 8 : (n <= 16384 ? 16 : 0);
}

int sk_transform_supported(int n, int storage, size_t max_lds) {
  const size_t elem = storage == 0 ? sizeof(double2) : sizeof(float2);
  return fft_values_per_thread(n, elem, max_lds) > 0 || n <= kMaxDirectDft;
}

template <typename T>
static hipError_t row_transform(const typename Cplx<T>::type* in, typename Cplx<T>::type* out,
                                int n, int rows, const typename Cplx<T>::type* tw, size_t max_lds,
                                hipStream_t st) {
  using V = typename Cplx<T>::type;
  const int E = fft_values_per_thread(n, sizeof(V), max_lds);
  if (E) {
    const int tpr = n / E;
    const int rpb = tpr >= 256 ? 1 : 256 / tpr;
    const size_t lds = (size_t)rpb * n * sizeof(V);
    const dim3 grid((rows + rpb - 1) / rpb), block(rpb * tpr);
    if (E == 8) {
      hipLaunchKernelGGL((fft_rows_kernel<T, 8>), grid, block, lds, st, in, out, n, ilog2(n),
                         rows, tw);
    } else {
      // 16 values per thread: rows of 16384, which only FP32 fits in LDS
      if constexpr (sizeof(T) == 4)
        hipLaunchKernelGGL((fft_rows_kernel<T, 16>), grid, block, lds, st, in, out, n,
                           ilog2(n), rows, tw);
      else
        return hipErrorInvalidValue;
    }
  } else {
    hipLaunchKernelGGL(dft_rows_kernel<T>, dim3((n + 127) / 128, rows), dim3(128), 0, st, in, out,
                       n, tw);
  }
  return hipGetLastError();
}

hipError_t sk_prepare(size_t max_lds) {
  const void* k[] = {(const void*)fft_rows_kernel<double, 8>, (const void*)fft_rows_kernel<float, 8>,
                     (const void*)fft_rows_kernel<float, 16>};
  for (const void* f : k) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
static hipError_t sk_sample_t(void* z, void* zt, double* acc, int nx, int ny, const void* twx,
                              const void* twy, size_t max_lds, hipStream_t st) {
  using V = typename Cplx<T>::type;
  V* a = (V*)z;
  V* b = (V*)zt;
  hipError_t e = row_transform<T>(a, b, nx, 2 * ny, (const V*)twx, max_lds, st);
  if (e != hipSuccess) return e;
  constexpr int TILE = kTransposeTile;
  hipLaunchKernelGGL(transpose_kernel<V>, dim3((nx + TILE - 1) / TILE, (ny + TILE - 1) / TILE, 2),
                     dim3(256), 0, st, b, a, ny, nx);
  e = row_transform<T>(a, b, ny, 2 * nx, (const V*)twy, max_lds, st);
  if (e != hipSuccess) return e;
  const uint32_t H = (uint32_t)(nx / 2 + 1) * ny;
  hipLaunchKernelGGL(sk_accumulate_kernel<T>, dim3((H + 255) / 256), dim3(256), 0, st, b, acc, nx,
                     ny);
  return hipGetLastError();
}

// One structure-factor sample.  z holds the planes the step kernel wrote
// ([2][ny][nx], storage precision) and is overwritten; zt is scratch of the
// same size; twx / twy are the twiddle tables (storage precision, nx and ny
// entries); acc: 5 (nx/2 + 1) ny FP64 accumulators, [which][kx][ky].
hipError_t launch_sk_sample(int storage, void* z, void* zt, double* acc, int nx, int ny,
                            const void* twx, const void* twy, size_t max_lds, hipStream_t st) {
  if (storage == 0) return sk_sample_t<double>(z, zt, acc, nx, ny, twx, twy, max_lds, st);
  return sk_sample_t<float>(z, zt, acc, nx, ny, twx, twy, max_lds, st);
}

}  // namespace flb
