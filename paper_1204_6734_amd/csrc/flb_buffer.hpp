// flb_buffer.hpp — device helpers shared by the D2Q9 and D3Q19 step kernels:
// raw buffer access to one population plane, the XCD-aware renumbering of
// workgroups and the wavefront reduction of the correlator sums.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace flb {

// Workgroups are dealt to the eight XCDs round-robin (workgroup b runs on
// XCD b mod 8).  Renumber them so that XCD k takes the k-th contiguous
// eighth of the nb work items, in order: neighbouring tiles, whose halos
// overlap, then share one XCD's L2.
__device__ __forceinline__ int xcd_tile(int bid, int nb) {
  const int q = nb >> 3, r = nb & 7, xcd = bid & 7;
  return xcd * q + (xcd < r ? xcd : r) + (bid >> 3);
}

// Raw buffer access to one population plane: the 128-bit resource (base,
// size) is wave-uniform and lives in SGPRs, the per-lane byte offset is a
// 32-bit VGPR and the wave-uniform row offset goes in the instruction's
// scalar offset operand, so no per-lane 64-bit address arithmetic is
// needed.  An offset outside the plane reads zero and drops the store.
// Planes must be smaller than 4 GiB.
template <typename S>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(void* pop, uint32_t N, int k) {
  char* base = reinterpret_cast<char*>(pop) + (size_t)k * N * sizeof(S);
  return __builtin_amdgcn_make_buffer_rsrc(base, 0, N * (uint32_t)sizeof(S), 0x00020000);
}

__device__ __forceinline__ float buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                          uint32_t soff, float*) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                           uint32_t soff, double*) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff,
                                          float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, 0);
}
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff,
                                          double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
}

// a where mask is all ones, b where it is zero (bitwise, so the choice is
// never turned into a dynamically indexed array access)
__device__ __forceinline__ double pick(uint64_t mask, double a, double b) {
  const uint64_t ua = __builtin_bit_cast(uint64_t, a), ub = __builtin_bit_cast(uint64_t, b);
  return __builtin_bit_cast(double, (ua & mask) | (ub & ~mask));
}

// One butterfly pass across 32 (W = 32) or 16 lanes on the value pair
// (a, b) = (v[k], v[k + n]): lanes whose bit W is clear keep a and add their
// partner's a, the others keep b and add their partner's b.  The gfx950 lane
// swap instructions move exactly these halves (per 32-bit word), so the pass
// needs no selects and no trip through the LDS crossbar.
template <int W>
__device__ __forceinline__ double swap_pass(double a, double b) {
  const uint64_t ua = __builtin_bit_cast(uint64_t, a), ub = __builtin_bit_cast(uint64_t, b);
  const uint32_t al = (uint32_t)ua, ah = (uint32_t)(ua >> 32);
  const uint32_t bl = (uint32_t)ub, bh = (uint32_t)(ub >> 32);
  uint32_t f0, f1, s0, s1;
  if constexpr (W == 32) {
    const auto lo = __builtin_amdgcn_permlane32_swap(al, bl, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(ah, bh, false, false);
    f0 = lo[0], s0 = lo[1], f1 = hi[0], s1 = hi[1];
  } else {
    static_assert(W == 16, "lane swaps exist across 32 and 16 lanes");
    const auto lo = __builtin_amdgcn_permlane16_swap(al, bl, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(ah, bh, false, false);
    f0 = lo[0], s0 = lo[1], f1 = hi[0], s1 = hi[1];
  }
  const double f = __builtin_bit_cast(double, ((uint64_t)f1 << 32) | f0);
  const double s = __builtin_bit_cast(double, ((uint64_t)s1 << 32) | s0);
  return f + s;
}

// Sums of 32 per-lane FP64 values over a 64-lane wavefront, transposed: five
// butterfly passes each halve the number of values a lane carries (lanes
// whose bit `off` is set keep the upper half) and a last pass adds the two
// lanes that share a value, after which lanes 2v and 2v+1 both hold the wave
// total of value v.  The passes across 32 and 16 lanes, which carry 24 of the
// 31 exchanges, use lane swaps; the narrow ones exchange through ds_bpermute.
__device__ __forceinline__ double wave_transpose_sum32(double (&v)[32], int lane) {
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = swap_pass<32>(v[k], v[k + 16]);
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = swap_pass<16>(v[k], v[k + 8]);
#pragma unroll
  for (int off = 8, n = 4; off >= 2; off >>= 1, n >>= 1) {
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

}  // namespace flb
