// flb_buffer.hpp — device helpers shared by the D2Q9 and D3Q19 step kernels:
// raw buffer access to one population plane and the XCD-aware renumbering of
// workgroups.
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

// The same for one row of a row-interleaved array (the nine plane rows of
// lattice row y, 9 pitch elements from element 9 y pitch): the plane goes in
// the scalar offset, the column in the per-lane offset.
template <typename S>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(void* pop, uint32_t pitch, int y) {
  char* base = reinterpret_cast<char*>(pop) + (size_t)y * 9 * pitch * sizeof(S);
  return __builtin_amdgcn_make_buffer_rsrc(base, 0, 9 * pitch * (uint32_t)sizeof(S), 0x00020000);
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

}  // namespace flb
