// flb_step.hip — the batched fluctuating collide-and-stream step of libflb
// for gfx950 (MI355X).
//
// step_kernel is one fused update (Kaehler & Wagner, Sec. II eq. (6) with the
// f-norm basis of Sec. IV) over every site of one or more lattices
// ("slots"), with the correlator sums of eqs. (16)/(23) and the
// structure-factor fields of eqs. (24)-(26) fused in when a sample is due.
//
// Memory layout: one population array per lattice of shifted values
// h_i = f_i - f_i^0(rho0, u0) (FP32 or FP64), row-interleaved (the nine plane
// rows of each lattice row together, see SlotDesc), updated
// in place with the two-phase "AA" access pattern: on even steps a site
// reads its own nine slots and writes the post-collision values back
// reversed; on odd steps it reads the reversed values of its neighbours and
// writes forward to its neighbours.  Each site touches the same nine
// locations it reads, so no second buffer is needed.  The unit of work is a
// tile of 256 sites, one wavefront per 64 consecutive sites of a row: 256 x 1
// (four wavefronts along a row) on rows of 256 sites or more, else 64 x 4
// (four rows).  A workgroup takes 1, 2 or 4 consecutive tiles
// ("tile group"), and the grid is either one workgroup per tile group or a
// smaller persistent grid striding over the tile groups; the autotuner picks
// among these shapes, which all compute bit-identical results.  Tile groups
// are renumbered so that each XCD (workgroups are dealt to the eight XCDs
// round-robin) sweeps a contiguous band of rows and keeps its halo rows in
// its own L2.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "flb_buffer.hpp"
#include "flb_device.hpp"
#include "flb_kernels.hpp"

namespace flb {

__device__ __forceinline__ int find_slot(const int* __restrict__ prefix, int nslots, int tile) {
  int lo = 0, hi = nslots;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= tile) lo = mid; else hi = mid;
  }
  return lo;
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
  C.xc2 = sd.xc2f;
  C.one_tau = sd.one_tau;
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
  C.xc2 = sd.xc2;
  C.one_tau = sd.one_tau;
  C.k0 = sd.k0;
  C.k1 = sd.k1;
  C.noise = sd.noise;
  return C;
}

typedef double double4_v __attribute__((ext_vector_type(4)));

// Position of statistic v in a wavefront's 16 x 16 result X^T X (row-major):
// the sum of df_i is entry (i, 9), the product df_i df_j (i <= j) entry (i, j).
struct StatPos {
  int pos[kNStat];
};
constexpr StatPos stat_positions() {
  StatPos p{};
  int q = 0;
  for (int i = 0; i < 9; ++i) p.pos[q++] = i * 16 + 9;
  for (int i = 0; i < 9; ++i)
    for (int j = i; j < 9; ++j) p.pos[q++] = i * 16 + j;
  return p;
}
__constant__ StatPos kStatPos = stat_positions();

typedef __bf16 bf16x8_v __attribute__((ext_vector_type(8)));
typedef float float4_v __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4_v __attribute__((ext_vector_type(4)));

// x = x1 + x2 + x3 exactly, each part a bfloat16 (returned as its 16 bits):
// x1 keeps the leading 8 significant bits of x (truncated), x2 the leading 8
// of what remains, x3 the rest, which has at most 8 significant bits left
// (an FP32 value has 24).  Both subtractions are exact.
__device__ __forceinline__ void split_bf16x3(float x, uint32_t p[3]) {
  const uint32_t b1 = __builtin_bit_cast(uint32_t, x) & 0xFFFF0000u;
  const float r1 = x - __builtin_bit_cast(float, b1);
  const uint32_t b2 = __builtin_bit_cast(uint32_t, r1) & 0xFFFF0000u;
  const float r2 = r1 - __builtin_bit_cast(float, b2);
  p[0] = b1 >> 16;
  p[1] = b2 >> 16;
  p[2] = __builtin_bit_cast(uint32_t, r2) >> 16;
}

// Correlator sums of df_i = f_i - f_i^0(rho0, u0) (= the stored h_i): 9
// first moments and the 45 products i <= j (row-major), added to this
// tile's open time-block partials.  For one wavefront (64 sites) these are
// the entries of X^T X, X the 64 x 10 matrix of the nine df_i and a
// constant 1 per site, a dense contraction over the sites done on the
// matrix cores; the wavefront stages its values in LDS first.
//   FP32 storage: every df_i is split exactly into three bfloat16 parts,
//   x = x1 + x2 + x3, so that x y = sum_{p,q} xp yq with every part product
//   exact in FP32; eighteen v_mfma_f32_16x16x32_bf16 (the nine part pairs,
//   32 sites each) accumulate the 16 x 16 result in FP32.  Operand layout:
//   lane l holds feature l % 16 of sites 8 (l / 16) .. + 7 of a group of 32
//   (the same registers serve as A and B); result row 4 (l / 16) + r,
//   column l % 16 in element r.  The products are exact and a wavefront's
//   sum of 64 sites has the rounding of FP32 additions (a few 1e-8
//   relative); all later sums are FP64.
//   FP64 storage: sixteen v_mfma_f64_16x16x4f64 (four sites each) on the
//   values themselves, lane l taking column l % 16 of site l / 16 of each
//   group of four; result row l / 16 + 4 r, column l % 16 in element r.
// The wavefront writes its 16 x 16 result (FP64) over its staged values;
// at the end of the step the four wavefronts of the tile add their results
// in a fixed order, so a tile's partial does not depend on the workgroup
// shape.
template <typename S>
constexpr int sample_wave_bytes() {
  // FP32: 3 parts x 10 values (the nine df_i and the constant) x 64 sites
  // of 2 bytes; FP64: 64 x 9 values; at least the 16 x 16 FP64 result
  return sizeof(S) == 4 ? 3 * 10 * kTileX * 2 : kTileX * 9 * 8;
}

// The staging areas of the workgroup's wavefronts: one per wavefront
// (dynamic LDS, sized at launch for the workgroup's tiles, so that one-tile
// workgroups keep their occupancy).
template <typename S>
__device__ __forceinline__ double* wave_staging(int sub, int wave) {
  extern __shared__ __attribute__((aligned(16))) double xs_dyn[];
  constexpr int kWaveDoubles = sample_wave_bytes<S>() / (int)sizeof(double);
  return xs_dyn + (sub * kTileY + wave) * kWaveDoubles;
}

// One wavefront's part: X^T X of its 64 sites into its staging area (no
// barrier).  Sites outside the lattice hold zeros in h.
template <typename S, typename R>
__device__ __forceinline__ void wave_correlators(const R h[9], int sub, int wave) {
  static_assert(sample_wave_bytes<S>() >= 16 * 16 * (int)sizeof(double),
                "the result fits the staging area");
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, grp = lane >> 4;
  double* out = wave_staging<S>(sub, wave);
  if constexpr (sizeof(S) == 4) {
    // staging [part 3][value 10][site 64] of bfloat16; value 9 is the
    // constant 1 = 1 + 0 + 0 (bfloat16 one is 0x3F80)
    unsigned short* xb = reinterpret_cast<unsigned short*>(out);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      uint32_t pp[3];
      split_bf16x3((float)h[i], pp);
#pragma unroll
      for (int q = 0; q < 3; ++q) xb[(q * 10 + i) * kTileX + lane] = (unsigned short)pp[q];
    }
    xb[9 * kTileX + lane] = 0x3F80;
    xb[19 * kTileX + lane] = 0;
    xb[29 * kTileX + lane] = 0;
    // the values come back from other lanes of the same wavefront, whose
    // LDS accesses complete in program order
    __builtin_amdgcn_wave_barrier();
    // rows 10..15 of the result are not used: those lanes read row 9
    const int colr = col < 10 ? col : 9;
    u32x4_v X[3][2];
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int hh = 0; hh < 2; ++hh)
        X[q][hh] = *reinterpret_cast<const u32x4_v*>(xb + (q * 10 + colr) * kTileX + 32 * hh +
                                                     8 * grp);
    // the result is written over the staged values: every read above is
    // issued first (the compiler may not move the writes before them)
    asm volatile("" ::: "memory");
    // X^T X = sum over part pairs (p, q) of X_p^T X_q, and the (q, p) term is
    // the transpose of the (p, q) one: A holds the pairs p = q, B those with
    // p < q, and the sum is A + B + B^T.  The pair (2, 2) is left out: its
    // products are below 2^-30 of the others', under the rounding of the
    // FP32 accumulators.  Ten products per wavefront, in a fixed order.
    float4_v acc = {0.f, 0.f, 0.f, 0.f}, accb = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      const bf16x8_v x0 = __builtin_bit_cast(bf16x8_v, X[0][hh]);
      const bf16x8_v x1 = __builtin_bit_cast(bf16x8_v, X[1][hh]);
      const bf16x8_v x2 = __builtin_bit_cast(bf16x8_v, X[2][hh]);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x0, x0, acc, 0, 0, 0);
      accb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x0, x1, accb, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x1, x1, acc, 0, 0, 0);
      accb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x0, x2, accb, 0, 0, 0);
      accb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x1, x2, accb, 0, 0, 0);
    }
    // B^T through LDS: B goes past the 2 KiB of the result, in the staging
    // area the operands were read from, and comes back transposed
    static_assert(sample_wave_bytes<S>() >= 2048 + 16 * 16 * (int)sizeof(float),
                  "B fits the staging area after the result");
    float* bt = reinterpret_cast<float*>(reinterpret_cast<char*>(out) + 2048);
#pragma unroll
    for (int r = 0; r < 4; ++r) bt[(4 * grp + r) * 16 + col] = accb[r];
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < 4; ++r)
      out[(4 * grp + r) * 16 + col] =
          (double)((acc[r] + accb[r]) + bt[col * 16 + 4 * grp + r]);
  } else {
    S* x = reinterpret_cast<S*>(out);
#pragma unroll
    for (int i = 0; i < 9; ++i) x[lane * 9 + i] = (S)h[i];
    __builtin_amdgcn_wave_barrier();
    // columns 10..15 are zero and column 9 is the constant; every lane reads
    // an in-range element so that the sixteen reads issue back to back
    const int colr = col < 9 ? col : 8;
    const double pad = col == 9 ? 1.0 : 0.0;
    S xv[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) xv[q] = x[(4 * q + grp) * 9 + colr];
    asm volatile("" ::: "memory");
    double4_v acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const double val = col < 9 ? (double)xv[q] : pad;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(val, val, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) out[(grp + 4 * r) * 16 + col] = acc[r];
  }
}

// The tile's part: after a workgroup barrier, 54 threads add the four
// wavefronts' results in a fixed order to the tile's partials.  Every
// thread of the workgroup calls this; `due` is uniform over one tile.  No
// second barrier: a sampling step gives every tile of a workgroup its own
// staging areas and is never persistent, so nothing reuses them.
template <typename S>
__device__ __forceinline__ void tile_correlators(bool due, double* __restrict__ partials,
                                                 int sub) {
  const int v = threadIdx.x & (kBlock - 1);
  const bool adds = due && v < kNStat;
  const int pos = adds ? kStatPos.pos[v] : 0;
  __syncthreads();
  if (adds) {
    const double tot = (wave_staging<S>(sub, 0)[pos] + wave_staging<S>(sub, 1)[pos]) +
                       (wave_staging<S>(sub, 2)[pos] + wave_staging<S>(sub, 3)[pos]);
    partials[v] += tot;
  }
}

// Where the nine populations a site reads in phase ODD are, in the
// row-interleaved storage: the row (a buffer resource of one lattice row,
// wave-uniform), the plane (the scalar offset, wave-uniform) and the column
// (the per-lane offset).  Even phase: plane i at the site itself.  Odd
// phase: plane opp(i) at x - v_i.  After the collision the value of
// direction kOpp[i] goes back to the same place.  A wavefront holds 64
// sites of one row, so only the x wrap is per lane, and only wavefronts at
// the two ends of a row can wrap.
template <typename S, int ODD>
__device__ __forceinline__ void site_offsets(void* pop, uint32_t pitch, int x, int y, int nx,
                                             int ny, bool x_edge, __amdgpu_buffer_rsrc_t rs[9],
                                             uint32_t voff[9], uint32_t soff[9]) {
  constexpr uint32_t E = sizeof(S);
  const uint32_t pe = pitch * E;  // bytes per plane row
  const uint32_t xc = (uint32_t)x * E;
  const __amdgpu_buffer_rsrc_t rc = row_rsrc<S>(pop, pitch, y);
  if (!ODD) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      rs[i] = rc;
      voff[i] = xc;
      soff[i] = (uint32_t)i * pe;
    }
  } else {
    const __amdgpu_buffer_rsrc_t rm = row_rsrc<S>(pop, pitch, y == 0 ? ny - 1 : y - 1);
    const __amdgpu_buffer_rsrc_t rp = row_rsrc<S>(pop, pitch, y == ny - 1 ? 0 : y + 1);
    uint32_t xm = xc - E, xp = xc + E;
    if (x_edge) {
      // a wave-uniform branch: the empty volatile asm keeps the compiler
      // from turning the wrap into selects that every wavefront would run
      asm volatile("" : "+v"(xm), "+v"(xp));
      xm = x == 0 ? (uint32_t)(nx - 1) * E : xm;
      xp = x == nx - 1 ? 0u : xp;
    }
    rs[0] = rc; voff[0] = xc;  // v=( 0, 0)
    rs[1] = rc; voff[1] = xm;  // v=( 1, 0) from (x-1, y)
    rs[2] = rm; voff[2] = xc;  // v=( 0, 1) from (x, y-1)
    rs[3] = rc; voff[3] = xp;  // v=(-1, 0) from (x+1, y)
    rs[4] = rp; voff[4] = xc;  // v=( 0,-1) from (x, y+1)
    rs[5] = rm; voff[5] = xm;  // v=( 1, 1) from (x-1, y-1)
    rs[6] = rm; voff[6] = xp;  // v=(-1, 1) from (x+1, y-1)
    rs[7] = rp; voff[7] = xp;  // v=(-1,-1) from (x+1, y+1)
    rs[8] = rp; voff[8] = xm;  // v=( 1,-1) from (x-1, y+1)
#pragma unroll
    for (int i = 0; i < 9; ++i) soff[i] = (uint32_t)kOpp[i] * pe;
  }
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
  // t < tend, as the sign of tend - t (both below 2^63; the scalar unit has
  // no 64-bit ordered compare)
  const uint64_t rem = sd.tend - t;
  const bool live = have && (int32_t)(uint32_t)(rem >> 32) >= 0 && rem != 0;
  if (!SAMPLE && !live) return;
  const int lt = tile - prefix[s];
  const int nx = sd.nx, ny = sd.ny;
  // lt / tiles_x by multiply-shift on the scalar unit
  const int ty = (int)(((uint64_t)(uint32_t)lt * sd.tx_magic) >> sd.tx_shift);
  const int tx = lt - ty * sd.tiles_x;
  // first column of this wavefront's 64 sites, and its row: a wide tile
  // lays its four wavefronts along one row, a narrow one stacks them
  const int xw = sd.wide ? tx * (kTileY * kTileX) + wave * kTileX : tx * kTileX;
  const int y = sd.wide ? ty : ty * kTileY + wave;
  const int x = xw + (threadIdx.x & (kTileX - 1));
  const bool active = live && (x < nx) && (y < ny);
  const uint32_t N = (uint32_t)nx * (uint32_t)ny;

  // The offsets are computed outside the per-lane branch (they are only
  // arithmetic): the row resources and plane offsets then stay wave-uniform
  // in scalar registers up to the stores, which need them there.  They are
  // those of the site clamped onto the lattice, so that the lanes and
  // wavefronts of a ragged last tile load a real site's values (which they
  // never use) and the plain step's loads need no branch.
  __amdgpu_buffer_rsrc_t rs[9];
  uint32_t voff[9], soff[9];
  site_offsets<S, ODD>(sd.pop, sd.pitch, x < nx ? x : nx - 1, y < ny ? y : ny - 1, nx, ny,
                       xw == 0 || xw + kTileX >= nx, rs, voff, soff);
  R h[9];
  if (!SAMPLE || active) {
#pragma unroll
    for (int i = 0; i < 9; ++i) h[i] = (R)buf_load(rs[i], voff[i], soff[i], (S*)nullptr);
  } else {
    // the correlator sums take the sites off the lattice as zeros
#pragma unroll
    for (int i = 0; i < 9; ++i) h[i] = R(0);
  }

  const CollideConst<R> C = collide_const<R>(sd);
  const uint32_t site = (uint32_t)y * (uint32_t)nx + (uint32_t)x;
  // the Gaussians need only the site and the step: drawn here, while the
  // loads are still in flight, they cover part of the load latency
  constexpr bool kNoise32 = sizeof(S) < sizeof(R);
  SiteDraw<R, kNoise32> draw;  // read by the collision only where drawn
  if (active && C.noise) site_draw<R, kNoise32>(C, site, t, draw);

  bool due = false;
  if (SAMPLE) {
    due = live && sd.sample_every > 0 &&
          multiple_of(t, (uint32_t)sd.sample_every, sd.se_magic, sd.se_shift);
    if (due) wave_correlators<S, R>(h, sub, wave);
    if (live && sd.skz != nullptr && sd.sk_every > 0 &&
        multiple_of(t, (uint32_t)sd.sk_every, sd.sk_magic, sd.sk_shift) && active) {
      // structure-factor fields in the f-norm at (rho0, u0): d rho and
      // dj~ = sqrt3 (j - u0 rho) = sqrt3 ((j - rho0 u0) - u0 (rho - rho0))  (eq. (34)),
      // packed as z1 = d rho + i dj~_x, z2 = dj~_y in the storage precision
      using V = typename Cplx<S>::type;
      double hd[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) hd[i] = (double)h[i];
      const Moments<double> m = hermite_moments(hd);
      V* z = reinterpret_cast<V*>(sd.skz);
      z[site] = V{(S)m.drho, (S)(1.7320508075688772935 * (m.jx - sd.ux0 * m.drho))};
      z[N + site] = V{(S)(1.7320508075688772935 * (m.jy - sd.uy0 * m.drho)), S(0)};
    }
  }

  if (active) {
    const int e = collide<R, BASIS, kNoise32>(h, C, draw);
    if (e) {
      atomicOr(sd.err, e);
      atomicMin(sd.err_step, (unsigned long long)t);
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) buf_store(rs[i], voff[i], soff[i], (S)h[kOpp[i]]);
  }
  // the tile's correlator sums last, so that its barrier does not hold the
  // wavefronts between their loads and their stores
  if (SAMPLE) tile_correlators<S>(due, sd.partials + (size_t)(due ? lt : 0) * kNStat, sub);
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

// The step's memory traffic with none of its arithmetic (a bandwidth
// probe): every site of an nx x ny lattice loads its nine values at phase
// ODD and stores them back as the step does, with the step's tiles,
// workgroup order and addressing.
template <typename S, int ODD>
__global__ __launch_bounds__(kBlock) void stream_probe_kernel(void* pop, int nx, int ny,
                                                              uint32_t pitch, int wide,
                                                              int tiles_x, int ntiles) {
  const int tile = xcd_tile(blockIdx.x, ntiles);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
  const int xw = wide ? tx * (kTileY * kTileX) + wave * kTileX : tx * kTileX;
  const int y = wide ? ty : ty * kTileY + wave;
  const int x = xw + (threadIdx.x & (kTileX - 1));
  if (x >= nx || y >= ny) return;
  __amdgpu_buffer_rsrc_t rs[9];
  uint32_t voff[9], soff[9];
  site_offsets<S, ODD>(pop, pitch, x, y, nx, ny, xw == 0 || xw + kTileX >= nx, rs, voff, soff);
  S h[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) h[i] = buf_load(rs[i], voff[i], soff[i], (S*)nullptr);
#pragma unroll
  for (int i = 0; i < 9; ++i) buf_store(rs[i], voff[i], soff[i], h[kOpp[i]]);
}

hipError_t launch_stream_probe(int storage, void* pop, int nx, int ny, uint32_t pitch, int wide,
                               int tiles_x, int ntiles, int odd, hipStream_t st) {
  const dim3 g(ntiles), b(kBlock);
#define FLB_PROBE(S)                                                                           \
  if (odd)                                                                                     \
    hipLaunchKernelGGL((stream_probe_kernel<S, 1>), g, b, 0, st, pop, nx, ny, pitch, wide,     \
                       tiles_x, ntiles);                                                       \
  else                                                                                         \
    hipLaunchKernelGGL((stream_probe_kernel<S, 0>), g, b, 0, st, pop, nx, ny, pitch, wide,     \
                       tiles_x, ntiles)
  if (storage == 0) FLB_PROBE(double);
  else FLB_PROBE(float);
#undef FLB_PROBE
  return hipGetLastError();
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
  const size_t lds = sample ? (size_t)tpb * kTileY * sample_wave_bytes<S>() : 0;
#define FLB_STEP(SMP, ODD, PER)                                                                   \
  hipLaunchKernelGGL((step_kernel<S, R, BASIS, SMP, ODD, PER>), g, b, lds, st, d_slots, d_prefix, \
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

}  // namespace flb
