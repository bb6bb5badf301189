// flb_kernels.hip — HIP kernels of libflb for gfx950 (MI355X).
//
// The hot kernel is step_kernel: one fused fluctuating collide-and-stream
// update (Kaehler & Wagner, Sec. II eq. (6) with the f-norm basis of
// Sec. IV) over every site of one or more lattices ("slots"), with the
// correlator sums of eqs. (16)/(23) and the structure-factor fields of
// eqs. (24)-(26) fused in when a sample is due.
//
// Memory layout: one population array per lattice, structure of arrays
// [9][ny][nx] of shifted values h_i = f_i - w_i rho0 (FP32 or FP64), updated
// in place with the two-phase "AA" access pattern: on even steps a site
// reads its own nine slots and writes the post-collision values back
// reversed; on odd steps it reads the reversed values of its neighbours and
// writes forward to its neighbours.  Each site touches the same nine
// locations it reads, so no second buffer is needed.  The unit of work is a
// 64 x 4 tile (256 threads, one wavefront per tile row: every wavefront reads
// and writes whole rows).  A workgroup takes 1, 2 or 4 consecutive tiles
// ("tile group"), and the grid is either one workgroup per tile group or a
// smaller persistent grid striding over the tile groups; the autotuner picks
// among these shapes, which all compute bit-identical results.  Tile groups
// are renumbered so that each XCD (workgroups are dealt to the eight XCDs
// round-robin) sweeps a contiguous band of rows and keeps its halo rows in
// its own L2.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "flb_device.hpp"
#include "flb_kernels.hpp"

namespace flb {

// Complex value of a real type.
template <typename T> struct Cplx;
template <> struct Cplx<double> { using type = double2; };
template <> struct Cplx<float> { using type = float2; };

__device__ __forceinline__ int xcd_tile(int bid, int nb) {
  const int q = nb >> 3, r = nb & 7, xcd = bid & 7;
  return xcd * q + (xcd < r ? xcd : r) + (bid >> 3);
}

__device__ __forceinline__ int find_slot(const int* __restrict__ prefix, int nslots, int tile) {
  int lo = 0, hi = nslots;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= tile) lo = mid; else hi = mid;
  }
  return lo;
}

// Element indices of the nine populations a site reads in phase `odd`.
// After the collision the value of direction kOpp[i] goes back to idx[i].
__device__ __forceinline__ void site_indices(int x, int y, int nx, int ny, int odd,
                                             uint32_t N, uint32_t idx[9]) {
  const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
  const uint32_t rc = (uint32_t)y * nx, rm = (uint32_t)ym * nx, rp = (uint32_t)yp * nx;
  const uint32_t c = rc + x;
  if (!odd) {
#pragma unroll
    for (int i = 0; i < 9; ++i) idx[i] = (uint32_t)i * N + c;
  } else {
    // plane opp(i) at x - v_i
    idx[0] = c;
    idx[1] = 3u * N + rc + xm;   // v=( 1, 0): plane 3 at (x-1, y)
    idx[2] = 4u * N + rm + x;    // v=( 0, 1): plane 4 at (x, y-1)
    idx[3] = 1u * N + rc + xp;   // v=(-1, 0): plane 1 at (x+1, y)
    idx[4] = 2u * N + rp + x;    // v=( 0,-1): plane 2 at (x, y+1)
    idx[5] = 7u * N + rm + xm;   // v=( 1, 1): plane 7 at (x-1, y-1)
    idx[6] = 8u * N + rm + xp;   // v=(-1, 1): plane 8 at (x+1, y-1)
    idx[7] = 5u * N + rp + xp;   // v=(-1,-1): plane 5 at (x+1, y+1)
    idx[8] = 6u * N + rp + xm;   // v=( 1,-1): plane 6 at (x-1, y+1)
  }
}

template <typename R>
__device__ __forceinline__ CollideConst<R> collide_const(const SlotDesc& sd);

template <>
__device__ __forceinline__ CollideConst<float> collide_const<float>(const SlotDesc& sd) {
  CollideConst<float> C;
  C.rho0 = sd.rho0f;
  C.ux0 = sd.ux0f;
  C.uy0 = sd.uy0f;
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    C.rt[a] = sd.rtf[a];
    C.xc[a] = sd.xcf[a];
  }
  C.k0 = sd.k0;
  C.k1 = sd.k1;
  C.noise = sd.noise;
  return C;
}

template <>
__device__ __forceinline__ CollideConst<double> collide_const<double>(const SlotDesc& sd) {
  CollideConst<double> C;
  C.rho0 = sd.rho0;
  C.ux0 = sd.ux0;
  C.uy0 = sd.uy0;
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    C.rt[a] = sd.rt[a];
    C.xc[a] = sd.xc[a];
  }
  C.k0 = sd.k0;
  C.k1 = sd.k1;
  C.noise = sd.noise;
  return C;
}

// Sums of 32 per-lane values over a 64-lane wavefront, transposed: five
// butterfly passes each halve the number of values a lane carries and a
// last pass adds the two lanes that share a value, after which lanes 2v and
// 2v+1 both hold the wave total of value v.
__device__ __forceinline__ double pick(uint64_t mask, double a, double b) {
  // a where mask is all ones, b where it is zero (bitwise, so the choice is
  // never turned into a dynamically indexed array access)
  const uint64_t ua = __builtin_bit_cast(uint64_t, a), ub = __builtin_bit_cast(uint64_t, b);
  return __builtin_bit_cast(double, (ua & mask) | (ub & ~mask));
}

__device__ __forceinline__ double wave_transpose_sum32(double (&v)[32], int lane) {
#pragma unroll
  for (int off = 32, n = 16; off >= 2; off >>= 1, n >>= 1) {
    const uint64_t up = (lane & off) ? ~0ull : 0ull;
#pragma unroll
    for (int k = 0; k < n; ++k) {
      const double send = pick(up, v[k], v[k + n]);
      const double keep = pick(up, v[k + n], v[k]);
      v[k] = keep + __shfl_xor(send, off, 64);
    }
  }
  return v[0] + __shfl_xor(v[0], 1, 64);
}

// Correlator sums of df_i = f_i - f_i^0(rho0, u0) (= the stored h_i): 9
// first moments and the 45 products i <= j (row-major), added to this
// tile's open time-block partials.  Reduced in two groups of 32 values to
// keep registers low.  Every thread of the workgroup calls this (it holds
// two workgroup barriers); `due` is uniform over one tile and says whether
// the tile samples at all.  The partial of a tile is always formed in the
// same order, whatever the workgroup shape.
template <typename R>
__device__ __forceinline__ void sample_correlators(const R h[9], bool active, bool due,
                                                   double* __restrict__ partials, int sub,
                                                   int wave) {
  __shared__ double red[kMaxTilesPerBlock][kTileY][kTileX];
  const int lane = threadIdx.x & 63;
  if (due) {
    double df[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) df[i] = active ? (double)h[i] : 0.0;
#pragma unroll
    for (int group = 0; group < 2; ++group) {
      double v[32];
      int k = 0, q = 0;
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        if (q >= group * 32 && q < group * 32 + 32) v[k++] = df[i];
        ++q;
      }
#pragma unroll
      for (int i = 0; i < 9; ++i)
#pragma unroll
        for (int j = i; j < 9; ++j) {
          if (q >= group * 32 && q < group * 32 + 32) v[k++] = df[i] * df[j];
          ++q;
        }
#pragma unroll
      for (; k < 32; ++k) v[k] = 0.0;
      const double tot = wave_transpose_sum32(v, lane);
      if ((lane & 1) == 0) red[sub][wave][group * 32 + (lane >> 1)] = tot;
    }
  }
  __syncthreads();
  const int v = threadIdx.x & (kBlock - 1);
  if (due && v < kNStat) {
    const double tot = (red[sub][0][v] + red[sub][1][v]) + (red[sub][2][v] + red[sub][3][v]);
    partials[v] += tot;
  }
  __syncthreads();  // red is reused by the next tile group of a persistent grid
}

// Byte offsets (within their planes) of the nine populations a site reads
// in phase ODD, with the plane each one lives in.  Even phase: plane i at
// the site itself.  Odd phase: plane opp(i) at x - v_i.  After the
// collision the value of direction kOpp[i] goes back to the same place.
// Rows are wave-uniform (one wavefront = 64 sites of one row), so only the
// x wrap is per lane.
template <typename S, int ODD>
__device__ __forceinline__ void site_offsets(int x, int y, int nx, int ny, uint32_t off[9]) {
  constexpr uint32_t E = sizeof(S);
  const uint32_t rc = (uint32_t)y * nx * E;
  const uint32_t xc = (uint32_t)x * E;
  if (!ODD) {
#pragma unroll
    for (int i = 0; i < 9; ++i) off[i] = rc + xc;
  } else {
    const uint32_t rm = (uint32_t)(y == 0 ? ny - 1 : y - 1) * nx * E;
    const uint32_t rp = (uint32_t)(y == ny - 1 ? 0 : y + 1) * nx * E;
    const uint32_t xm = x == 0 ? (uint32_t)(nx - 1) * E : xc - E;
    const uint32_t xp = x == nx - 1 ? 0u : xc + E;
    off[0] = rc + xc;
    off[1] = rc + xm;  // v=( 1, 0) from (x-1, y)
    off[2] = rm + xc;  // v=( 0, 1) from (x, y-1)
    off[3] = rc + xp;  // v=(-1, 0) from (x+1, y)
    off[4] = rp + xc;  // v=( 0,-1) from (x, y+1)
    off[5] = rm + xm;  // v=( 1, 1) from (x-1, y-1)
    off[6] = rm + xp;  // v=(-1, 1) from (x+1, y-1)
    off[7] = rp + xp;  // v=(-1,-1) from (x+1, y+1)
    off[8] = rp + xm;  // v=( 1,-1) from (x-1, y+1)
  }
}

// Raw buffer access to one population plane: the 128-bit resource (base,
// size) is wave-uniform and lives in SGPRs, the per-lane byte offset is a
// 32-bit VGPR, so no per-lane 64-bit address arithmetic is needed.  An
// offset outside the plane reads zero and drops the store.
template <typename S>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(void* pop, uint32_t N, int k) {
  char* base = reinterpret_cast<char*>(pop) + (size_t)k * N * sizeof(S);
  return __builtin_amdgcn_make_buffer_rsrc(base, 0, N * (uint32_t)sizeof(S), 0x00020000);
}

__device__ __forceinline__ float buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off, float*) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off, double*) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, 0);
}
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, uint32_t off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
}

// One tile (or none: tile < 0) of the batched step.  A tile of a slot whose
// own time has reached its end is skipped; with SAMPLE the caller's whole
// workgroup still passes the barriers of the correlator reduction.
template <typename S, typename R, int BASIS, bool SAMPLE, int ODD>
__device__ __forceinline__ void step_tile(const SlotDesc* __restrict__ slots,
                                          const int* __restrict__ prefix, int nslots, int tile,
                                          uint64_t clk, int sub, int wave) {
  const bool have = tile >= 0;
  const int s = have ? find_slot(prefix, nslots, tile) : 0;
  const SlotDesc& sd = slots[s];
  const uint64_t t = sd.t0 + clk;
  const bool live = have && t < sd.tend;
  if (!SAMPLE && !live) return;
  const int lt = tile - prefix[s];
  const int nx = sd.nx, ny = sd.ny;
  const int ty = lt / sd.tiles_x, tx = lt - ty * sd.tiles_x;
  const int x = tx * kTileX + (threadIdx.x & (kTileX - 1));
  const int y = ty * kTileY + wave;
  const bool active = live && (x < nx) && (y < ny);
  const uint32_t N = (uint32_t)nx * (uint32_t)ny;

  uint32_t off[9];
  R h[9];
  if (active) {
    site_offsets<S, ODD>(x, y, nx, ny, off);
#pragma unroll
    for (int i = 0; i < 9; ++i)
      h[i] = (R)buf_load(plane_rsrc<S>(sd.pop, N, ODD ? kOpp[i] : i), off[i], (S*)nullptr);
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) h[i] = R(0);
  }

  if (SAMPLE) {
    const bool due = live && sd.sample_every > 0 && t % (uint64_t)sd.sample_every == 0;
    sample_correlators<R>(h, active, due, sd.partials + (size_t)(due ? lt : 0) * kNStat, sub,
                          wave);
    if (live && sd.skz != nullptr && sd.sk_every > 0 && t % (uint64_t)sd.sk_every == 0 &&
        active) {
      // structure-factor fields in the f-norm at (rho0, u0): d rho and
      // dj~ = sqrt3 (j - u0 rho) = sqrt3 ((j - rho0 u0) - u0 (rho - rho0))  (eq. (34)),
      // packed as z1 = d rho + i dj~_x, z2 = dj~_y in the storage precision
      using V = typename Cplx<S>::type;
      double hd[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) hd[i] = (double)h[i];
      const Moments<double> m = hermite_moments(hd);
      const uint32_t site = (uint32_t)y * nx + x;
      V* z = reinterpret_cast<V*>(sd.skz);
      z[site] = V{(S)m.drho, (S)(1.7320508075688772935 * (m.jx - sd.ux0 * m.drho))};
      z[N + site] = V{(S)(1.7320508075688772935 * (m.jy - sd.uy0 * m.drho)), S(0)};
    }
  }

  if (!active) return;
  const CollideConst<R> C = collide_const<R>(sd);
  const uint32_t site = (uint32_t)y * (uint32_t)nx + (uint32_t)x;
  const int e = collide<R, BASIS>(h, C, site, t);
  if (e) {
    atomicOr(sd.err, e);
    atomicMin(sd.err_step, (unsigned long long)t);
  }
#pragma unroll
  for (int i = 0; i < 9; ++i)
    buf_store(plane_rsrc<S>(sd.pop, N, ODD ? kOpp[i] : i), off[i], (S)h[kOpp[i]]);
}

// Tiles per workgroup a step variant accepts: the sampling variants and the
// FP64-compute variants need more than 128 registers, so they take at most
// two (a 1024-thread workgroup caps a thread at 128).
template <typename R, bool SAMPLE>
constexpr int max_tiles_per_block() {
  return (SAMPLE || sizeof(R) == 8) ? 2 : kMaxTilesPerBlock;
}

// The batched step: blockDim.x / 256 tiles per workgroup.  Without PERSIST
// workgroup b takes tile group b; with PERSIST (a grid smaller than the
// number of tile groups, and a multiple of eight so that a tile group stays
// on the XCD its renumbering assumes) it takes tile groups b, b + gridDim.x,
// ...  Only non-sampling steps run persistent (a loop around the reduction
// doubles its register use), and the one-group-per-workgroup variant keeps
// no loop at all, which measured about 3 % faster on the large lattice.
template <typename S, typename R, int BASIS, bool SAMPLE, int ODD, bool PERSIST>
__global__ __launch_bounds__((kBlock * max_tiles_per_block<R, SAMPLE>())) void step_kernel(
    const SlotDesc* __restrict__ slots, const int* __restrict__ prefix, int nslots,
    int total_tiles, const uint64_t* __restrict__ clock, uint32_t step_idx) {
  static_assert(!(SAMPLE && PERSIST), "sampling steps are not persistent");
  const int lg = blockDim.x >> 9;  // log2 of the tiles per workgroup
  const int ngroups = (total_tiles + (1 << lg) - 1) >> lg;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int sub = wid >> 2, wave = wid & (kTileY - 1);
  const uint64_t clk = *clock + step_idx;
  if (!PERSIST) {
    const int tile = (xcd_tile(blockIdx.x, ngroups) << lg) + sub;
    step_tile<S, R, BASIS, SAMPLE, ODD>(slots, prefix, nslots, tile < total_tiles ? tile : -1,
                                        clk, sub, wave);
  } else {
    for (int gb = blockIdx.x; gb < ngroups; gb += gridDim.x) {
      const int tile = (xcd_tile(gb, ngroups) << lg) + sub;
      step_tile<S, R, BASIS, false, ODD>(slots, prefix, nslots,
                                         tile < total_tiles ? tile : -1, clk, sub, wave);
    }
  }
}

__global__ void tick_kernel(uint64_t* clock, uint64_t n) { *clock += n; }

// ---------------------------------------------------------------- state I/O
// Write f (unshifted FP64, natural order, [9][ny][nx]) into storage at phase
// `odd` (odd: the reversed, un-streamed layout the next odd step reads).
template <typename S>
__global__ void write_state_kernel(S* pop, const double* __restrict__ f, int nx, int ny,
                                   int odd, Shift9 sh, int y0, int rows) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = y0 + (int)blockIdx.y;
  if (x >= nx) return;
  const uint32_t B = (uint32_t)nx * rows, bs = (uint32_t)blockIdx.y * nx + x;
  const uint32_t N = (uint32_t)nx * ny, site = (uint32_t)y * nx + x;
  uint32_t idx[9];
  site_indices(x, y, nx, ny, odd, N, idx);
#pragma unroll
  for (int i = 0; i < 9; ++i) pop[idx[i]] = (S)(f[i * (size_t)B + bs] - sh.v[i]);
  (void)site;
}

template <typename S>
__global__ void read_state_kernel(const S* __restrict__ pop, double* f, int nx, int ny, int odd,
                                  Shift9 sh, int y0, int rows) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = y0 + (int)blockIdx.y;
  if (x >= nx) return;
  const uint32_t B = (uint32_t)nx * rows, bs = (uint32_t)blockIdx.y * nx + x;
  const uint32_t N = (uint32_t)nx * ny, site = (uint32_t)y * nx + x;
  uint32_t idx[9];
  site_indices(x, y, nx, ny, odd, N, idx);
#pragma unroll
  for (int i = 0; i < 9; ++i) f[i * (size_t)B + bs] = (double)pop[idx[i]] + sh.v[i];
  (void)site;
}

// Raw storage copy in natural (even-phase) order for checkpoints: keeps the
// stored bits exactly.
template <typename S>
__global__ void raw_state_kernel(S* pop, S* buf, int nx, int ny, int odd, int to_buf, int y0,
                                 int rows) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = y0 + (int)blockIdx.y;
  if (x >= nx) return;
  const uint32_t B = (uint32_t)nx * rows, bs = (uint32_t)blockIdx.y * nx + x;
  const uint32_t N = (uint32_t)nx * ny, site = (uint32_t)y * nx + x;
  uint32_t idx[9];
  site_indices(x, y, nx, ny, odd, N, idx);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    if (to_buf) buf[i * (size_t)B + bs] = pop[idx[i]];
    else pop[idx[i]] = buf[i * (size_t)B + bs];
  }
  (void)site;
}

// Equilibrium f^0(rho(x), u(x)) from per-site fields (or uniform values when
// the field pointers are null), optionally plus ideal-gas fluctuations
// sqrt(mu f^0_i) N_i drawn with the thermal tag (two draws per site:
// step field 0 gives N_0..N_5, step field 1 gives N_6..N_8).
template <typename S>
__global__ void init_kernel(S* pop, const double* __restrict__ rho, const double* __restrict__ ux,
                            const double* __restrict__ uy, double rho0, double ux0, double uy0,
                            Shift9 sh, int nx, int ny, double mu, uint32_t k0, uint32_t k1,
                            int odd, int y0, int rows) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = y0 + (int)blockIdx.y;
  if (x >= nx) return;
  const uint32_t bs = (uint32_t)blockIdx.y * nx + x;  // index into band fields
  (void)rows;
  const uint32_t N = (uint32_t)nx * ny, site = (uint32_t)y * nx + x;
  const double r = rho ? rho[bs] : rho0;
  const double vx = ux ? ux[bs] : ux0, vy = uy ? uy[bs] : uy0;
  double g[9];
  unit_equilibrium(vx, vy, g);
  double n9[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (mu > 0.0) {
    double a[6], b[6];
    site_gaussians<double>(k0, k1, site, 0, 0x80000000u, a);
    site_gaussians<double>(k0, k1, site, 1, 0x80000000u, b);
    for (int i = 0; i < 6; ++i) n9[i] = a[i];
    for (int i = 0; i < 3; ++i) n9[6 + i] = b[i];
  }
  uint32_t idx[9];
  site_indices(x, y, nx, ny, odd, N, idx);
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
__global__ void moments_kernel(const S* __restrict__ pop, const double* __restrict__ B,
                               double* out, int nx, int ny, int odd, double rho0, double ux0,
                               double uy0, Shift9 sh, int* err, int y0, int rows) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = y0 + (int)blockIdx.y;
  if (x >= nx) return;
  const uint32_t Bn = (uint32_t)nx * rows, bs = (uint32_t)blockIdx.y * nx + x;
  const uint32_t N = (uint32_t)nx * ny;
  uint32_t idx[9];
  site_indices(x, y, nx, ny, odd, N, idx);
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
template <typename S>
__global__ void fourier_mode_kernel(const S* __restrict__ pop, double2* partial, int nx, int ny,
                                    int odd, int which, int kx, int ky, double rho0, double ux0,
                                    double uy0) {
  __shared__ double sr[256], si[256];
  const int tid = threadIdx.x;
  const uint32_t N = (uint32_t)nx * ny;
  double ar = 0.0, ai = 0.0;
  for (uint32_t site = blockIdx.x * 256u + tid; site < N; site += gridDim.x * 256u) {
    const int y = (int)(site / (uint32_t)nx), x = (int)(site - (uint32_t)y * nx);
    uint32_t idx[9];
    site_indices(x, y, nx, ny, odd, N, idx);
    double h[9];
    for (int i = 0; i < 9; ++i) h[i] = (double)pop[idx[i]];
    const Moments<double> m = hermite_moments(h);
    double a = m.drho;
    if (which == 1) a = 1.7320508075688772935 * (m.jx - ux0 * m.drho);
    if (which == 2) a = 1.7320508075688772935 * (m.jy - uy0 * m.drho);
    (void)rho0;
    const long long px = ((long long)kx * x) % nx, py = ((long long)ky * y) % ny;
    const double ph = 2.0 * ((double)px / nx + (double)py / ny);
    double sn, cs;
    sincospi(ph, &sn, &cs);
    ar += a * cs;
    ai -= a * sn;
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
  if (tid == 0) partial[blockIdx.x] = make_double2(sr[0], si[0]);
}

// ------------------------------------------------------------ time blocks
// Close the open time block of a lattice: record[slot] = sum over tiles of
// the partials (fixed order), then clear the partials.
__global__ void close_block_kernel(double* partials, int ntiles, double* record) {
  const int v = threadIdx.x;
  if (v >= kNStat) return;
  double s = 0.0;
  for (int t = 0; t < ntiles; ++t) {
    s += partials[(size_t)t * kNStat + v];
    partials[(size_t)t * kNStat + v] = 0.0;
  }
  record[v] = s;
}

// Neighbouring records merge pairwise: rec[b] = rec[2b] + rec[2b+1].
__global__ void merge_blocks_kernel(double* rec, int nhalf) {
  const int v = threadIdx.x;
  if (v >= kNStat) return;
  for (int b = 0; b < nhalf; ++b)
    rec[(size_t)b * kNStat + v] = rec[(size_t)(2 * b) * kNStat + v] +
                                  rec[(size_t)(2 * b + 1) * kNStat + v];
}

// Sum of the open partials (fixed order) into out[kNStat].
__global__ void open_sum_kernel(const double* partials, int ntiles, double* out) {
  const int v = threadIdx.x;
  if (v >= kNStat) return;
  double s = 0.0;
  for (int t = 0; t < ntiles; ++t) s += partials[(size_t)t * kNStat + v];
  out[v] = s;
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

template <int R, int E, typename V>
__device__ __forceinline__ void pass_compute(V (&a)[E], int n, int t, int Ns,
                                             const V* __restrict__ tw) {
  const int tpr = n / E;
#pragma unroll
  for (int m = 0; m < E / R; ++m) {
    if (Ns > 1) {
      const int j = t + m * tpr;
      const int step = (j & (Ns - 1)) * (n / (Ns * R));
#pragma unroll
      for (int r = 1; r < R; ++r) a[m * R + r] = cmul(a[m * R + r], tw[r * step]);
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
// through TILE x TILE tiles in LDS (256 threads; 32 for double2, 64 for
// float2, 16 KB or 32 KB of LDS).
template <typename V>
__global__ __launch_bounds__(256) void transpose_kernel(const V* __restrict__ in, V* out,
                                                        int rows, int cols) {
  constexpr int TILE = sizeof(V) == 16 ? 32 : 64, STEP = 256 / TILE;
  __shared__ V tile[TILE][TILE + 1];
  const int bx = blockIdx.x * TILE, by = blockIdx.y * TILE;
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

// ------------------------------------------------------------ launchers
template <typename S, typename R, int BASIS>
static hipError_t launch_step_t(bool sample, int odd, const SlotDesc* d_slots,
                                const int* d_prefix, int nslots, int total_tiles,
                                const uint64_t* d_clock, uint32_t step_idx, LaunchCfg cfg,
                                hipStream_t st) {
  if (total_tiles <= 0) return hipSuccess;
  if (cfg.tiles_per_block != 1 && cfg.tiles_per_block != 2 && cfg.tiles_per_block != 4)
    return hipErrorInvalidValue;
  if (cfg.grid_blocks < 0 || cfg.grid_blocks % 8 != 0) return hipErrorInvalidValue;
  const int tpb = std::min(cfg.tiles_per_block, sample ? max_tiles_per_block<R, true>()
                                                       : max_tiles_per_block<R, false>());
  const int ngroups = (total_tiles + tpb - 1) / tpb;
  const int grid =
      !sample && cfg.grid_blocks > 0 && cfg.grid_blocks < ngroups ? cfg.grid_blocks : ngroups;
  const dim3 g(grid), b(kBlock * tpb);
#define FLB_STEP(SMP, ODD, PER)                                                                 \
  hipLaunchKernelGGL((step_kernel<S, R, BASIS, SMP, ODD, PER>), g, b, 0, st, d_slots, d_prefix, \
                     nslots, total_tiles, d_clock, step_idx)
  if (sample) {
    if (odd) FLB_STEP(true, 1, false);
    else FLB_STEP(true, 0, false);
  } else if (grid < ngroups) {
    if (odd) FLB_STEP(false, 1, true);
    else FLB_STEP(false, 0, true);
  } else {
    if (odd) FLB_STEP(false, 1, false);
    else FLB_STEP(false, 0, false);
  }
#undef FLB_STEP
  return hipGetLastError();
}

template <typename S, typename R>
static hipError_t launch_step_b(int basis, bool sample, int odd, const SlotDesc* a, const int* b,
                                int c, int d, const uint64_t* e, uint32_t f, LaunchCfg cfg,
                                hipStream_t g) {
  switch (basis) {
    case kBasisFnormLocal:
      return launch_step_t<S, R, kBasisFnormLocal>(sample, odd, a, b, c, d, e, f, cfg, g);
    case kBasisHermite:
      return launch_step_t<S, R, kBasisHermite>(sample, odd, a, b, c, d, e, f, cfg, g);
    case kBasisFnormLut:
      return launch_step_t<S, R, kBasisFnormLut>(sample, odd, a, b, c, d, e, f, cfg, g);
  }
  return hipErrorInvalidValue;
}

// storage: 0 = FP64, 1 = FP32 shifted; compute: 0 = FP64, 1 = FP32; odd: the
// streaming phase, which every slot of the launch shares (own time parity).
hipError_t launch_step(int storage, int compute, int basis, bool sample, int odd,
                       const SlotDesc* d_slots, const int* d_prefix, int nslots,
                       int total_tiles, const uint64_t* d_clock, uint32_t step_idx,
                       LaunchCfg cfg, hipStream_t st) {
  if (storage == 0)
    return launch_step_b<double, double>(basis, sample, odd, d_slots, d_prefix, nslots,
                                         total_tiles, d_clock, step_idx, cfg, st);
  if (compute == 0)
    return launch_step_b<float, double>(basis, sample, odd, d_slots, d_prefix, nslots,
                                        total_tiles, d_clock, step_idx, cfg, st);
  return launch_step_b<float, float>(basis, sample, odd, d_slots, d_prefix, nslots, total_tiles,
                                     d_clock, step_idx, cfg, st);
}

hipError_t launch_tick(uint64_t* d_clock, uint64_t n, hipStream_t st) {
  hipLaunchKernelGGL(tick_kernel, dim3(1), dim3(1), 0, st, d_clock, n);
  return hipGetLastError();
}

static dim3 row_grid(int nx, int rows) { return dim3((nx + 255) / 256, rows); }

// The row-parallel utility kernels below process the band of rows
// [y0, y0 + rows); their host-side arrays hold that band only.
hipError_t launch_write_state(int storage, void* pop, const double* f, int nx, int ny, int odd,
                              const Shift9& sh, int y0, int rows, hipStream_t st) {
  if (storage == 0)
    hipLaunchKernelGGL(write_state_kernel<double>, row_grid(nx, rows), dim3(256), 0, st,
                       (double*)pop, f, nx, ny, odd, sh, y0, rows);
  else
    hipLaunchKernelGGL(write_state_kernel<float>, row_grid(nx, rows), dim3(256), 0, st,
                       (float*)pop, f, nx, ny, odd, sh, y0, rows);
  return hipGetLastError();
}

hipError_t launch_read_state(int storage, const void* pop, double* f, int nx, int ny, int odd,
                             const Shift9& sh, int y0, int rows, hipStream_t st) {
  if (storage == 0)
    hipLaunchKernelGGL(read_state_kernel<double>, row_grid(nx, rows), dim3(256), 0, st,
                       (const double*)pop, f, nx, ny, odd, sh, y0, rows);
  else
    hipLaunchKernelGGL(read_state_kernel<float>, row_grid(nx, rows), dim3(256), 0, st,
                       (const float*)pop, f, nx, ny, odd, sh, y0, rows);
  return hipGetLastError();
}

hipError_t launch_raw_state(int storage, void* pop, void* buf, int nx, int ny, int odd,
                            int to_buf, int y0, int rows, hipStream_t st) {
  if (storage == 0)
    hipLaunchKernelGGL(raw_state_kernel<double>, row_grid(nx, rows), dim3(256), 0, st,
                       (double*)pop, (double*)buf, nx, ny, odd, to_buf, y0, rows);
  else
    hipLaunchKernelGGL(raw_state_kernel<float>, row_grid(nx, rows), dim3(256), 0, st,
                       (float*)pop, (float*)buf, nx, ny, odd, to_buf, y0, rows);
  return hipGetLastError();
}

hipError_t launch_init(int storage, void* pop, const double* rho, const double* ux,
                       const double* uy, double rho0, double ux0, double uy0, const Shift9& sh,
                       int nx, int ny, double mu, uint32_t k0, uint32_t k1, int odd, int y0,
                       int rows, hipStream_t st) {
  if (storage == 0)
    hipLaunchKernelGGL(init_kernel<double>, row_grid(nx, rows), dim3(256), 0, st, (double*)pop,
                       rho, ux, uy, rho0, ux0, uy0, sh, nx, ny, mu, k0, k1, odd, y0, rows);
  else
    hipLaunchKernelGGL(init_kernel<float>, row_grid(nx, rows), dim3(256), 0, st, (float*)pop,
                       rho, ux, uy, rho0, ux0, uy0, sh, nx, ny, mu, k0, k1, odd, y0, rows);
  return hipGetLastError();
}

hipError_t launch_moments(int storage, const void* pop, const double* B, double* out, int nx,
                          int ny, int odd, double rho0, double ux0, double uy0,
                          const Shift9& sh, int* err, int y0, int rows, hipStream_t st) {
  if (storage == 0)
    hipLaunchKernelGGL(moments_kernel<double>, row_grid(nx, rows), dim3(256), 0, st,
                       (const double*)pop, B, out, nx, ny, odd, rho0, ux0, uy0, sh, err, y0,
                       rows);
  else
    hipLaunchKernelGGL(moments_kernel<float>, row_grid(nx, rows), dim3(256), 0, st,
                       (const float*)pop, B, out, nx, ny, odd, rho0, ux0, uy0, sh, err, y0,
                       rows);
  return hipGetLastError();
}

hipError_t launch_fourier_mode(int storage, const void* pop, double2* partial, int nblocks,
                               int nx, int ny, int odd, int which, int kx, int ky, double rho0,
                               double ux0, double uy0, hipStream_t st) {
  if (storage == 0)
    hipLaunchKernelGGL(fourier_mode_kernel<double>, dim3(nblocks), dim3(256), 0, st,
                       (const double*)pop, partial, nx, ny, odd, which, kx, ky, rho0, ux0, uy0);
  else
    hipLaunchKernelGGL(fourier_mode_kernel<float>, dim3(nblocks), dim3(256), 0, st,
                       (const float*)pop, partial, nx, ny, odd, which, kx, ky, rho0, ux0, uy0);
  return hipGetLastError();
}

hipError_t launch_close_block(double* partials, int ntiles, double* record, hipStream_t st) {
  hipLaunchKernelGGL(close_block_kernel, dim3(1), dim3(64), 0, st, partials, ntiles, record);
  return hipGetLastError();
}

hipError_t launch_merge_blocks(double* rec, int nhalf, hipStream_t st) {
  hipLaunchKernelGGL(merge_blocks_kernel, dim3(1), dim3(64), 0, st, rec, nhalf);
  return hipGetLastError();
}

hipError_t launch_open_sum(const double* partials, int ntiles, double* out, hipStream_t st) {
  hipLaunchKernelGGL(open_sum_kernel, dim3(1), dim3(64), 0, st, partials, ntiles, out);
  return hipGetLastError();
}

hipError_t launch_fill(double* p, size_t n, double v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
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
  constexpr int TILE = sizeof(V) == 16 ? 32 : 64;
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
