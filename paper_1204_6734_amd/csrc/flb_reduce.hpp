// flb_reduce.hpp — reductions of the per-tile correlator partials
// ([ntiles][NSTAT] FP64 sums, one row per tile) into a time-block record or
// the open sums, shared by the D2Q9 (54 statistics) and D3Q19 (209) paths.
// The order of every addition depends only on the tile count, so a lattice
// gives the same sums whatever else runs and however it was launched.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace flb {

// Thread layout (v, j): v = statistic (padded to VP), j = one of J lanes
// over the tiles.
template <int NSTAT>
struct SumShape {
  static constexpr int VP = NSTAT <= 64 ? 64 : 256;
  static constexpr int J = 1024 / VP;
};

// Stage one of closing a block: workgroup b sums tiles [b c, min((b+1) c, n))
// (lane j takes every J-th tile, then the J lane sums are added in order),
// writes the sum into the range's first row and clears the others.
template <int NSTAT>
__device__ __forceinline__ void fold_tiles(double* partials, int ntiles, int chunk) {
  constexpr int VP = SumShape<NSTAT>::VP, J = SumShape<NSTAT>::J;
  __shared__ double red[J][VP];
  const int v = threadIdx.x % VP, j = threadIdx.x / VP;
  const int t0 = blockIdx.x * chunk, t1 = min(t0 + chunk, ntiles);
  double s = 0.0;
  if (v < NSTAT) {
    for (int t = t0 + j; t < t1; t += J) {
      double* q = partials + (size_t)t * NSTAT + v;
      s += *q;
      if (t != t0) *q = 0.0;
    }
  }
  red[j][v] = s;
  __syncthreads();
  if (j == 0 && v < NSTAT) {
    double tot = red[0][v];
#pragma unroll
    for (int k = 1; k < J; ++k) tot += red[k][v];
    partials[(size_t)t0 * NSTAT + v] = tot;
  }
}

// Stage two: record = the folded rows summed in range order; rows cleared.
template <int NSTAT>
__device__ __forceinline__ void gather_folds(double* partials, int nranges, int chunk,
                                             double* record) {
  const int v = threadIdx.x;
  if (v >= NSTAT) return;
  double s = 0.0;
  for (int b = 0; b < nranges; ++b) {
    double* q = partials + (size_t)b * chunk * NSTAT + v;
    s += *q;
    *q = 0.0;
  }
  record[v] = s;
}

template <int NSTAT>
__global__ __launch_bounds__(1024) void fold_tiles_kernel(double* partials, int ntiles,
                                                          int chunk) {
  fold_tiles<NSTAT>(partials, ntiles, chunk);
}

template <int NSTAT>
__global__ void gather_folds_kernel(double* partials, int nranges, int chunk, double* record) {
  gather_folds<NSTAT>(partials, nranges, chunk, record);
}

// The same two stages for several lattices of one tile count at once, the
// lattice in blockIdx.y: each one's sums are added in the order above.
template <int NSTAT>
__global__ __launch_bounds__(1024) void fold_tiles_many_kernel(double* const* partials, int ntiles,
                                                               int chunk) {
  fold_tiles<NSTAT>(partials[blockIdx.y], ntiles, chunk);
}

template <int NSTAT>
__global__ void gather_folds_many_kernel(double* const* partials, int nranges, int chunk,
                                         double* const* records, size_t record_offset) {
  gather_folds<NSTAT>(partials[blockIdx.y], nranges, chunk, records[blockIdx.y] + record_offset);
}

// Open sums (partials left as they are): one workgroup, lanes as above.
template <int NSTAT>
__global__ __launch_bounds__(1024) void open_sums_kernel(const double* partials, int ntiles,
                                                         double* out) {
  constexpr int VP = SumShape<NSTAT>::VP, J = SumShape<NSTAT>::J;
  __shared__ double red[J][VP];
  const int v = threadIdx.x % VP, j = threadIdx.x / VP;
  double s = 0.0;
  if (v < NSTAT)
    for (int t = j; t < ntiles; t += J) s += partials[(size_t)t * NSTAT + v];
  red[j][v] = s;
  __syncthreads();
  if (j == 0 && v < NSTAT) {
    double tot = red[0][v];
#pragma unroll
    for (int k = 1; k < J; ++k) tot += red[k][v];
    out[v] = tot;
  }
}

// Ranges of stage one: at most 256 workgroups of at least one tile.
inline void fold_ranges(int ntiles, int* chunk, int* nranges) {
  const int c = ntiles > 256 ? (ntiles + 255) / 256 : 1;
  *chunk = c;
  *nranges = (ntiles + c - 1) / c;
}

// record[NSTAT] = sum of the partials over all tiles; partials cleared.
template <int NSTAT>
hipError_t close_block_sums(double* partials, int ntiles, double* record, hipStream_t st) {
  if (ntiles <= 0) return hipErrorInvalidValue;
  int chunk = 1, nranges = 1;
  fold_ranges(ntiles, &chunk, &nranges);
  hipLaunchKernelGGL(fold_tiles_kernel<NSTAT>, dim3(nranges), dim3(1024), 0, st, partials,
                     ntiles, chunk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gather_folds_kernel<NSTAT>, dim3(1), dim3(SumShape<NSTAT>::VP), 0, st,
                     partials, nranges, chunk, record);
  return hipGetLastError();
}

// For n lattices of ntiles tiles each (device arrays of their partials and
// record bases): records[k] + record_offset = lattice k's sums; its
// partials cleared.  The same sums as close_block_sums for each.
template <int NSTAT>
hipError_t close_block_sums_many(double* const* partials, double* const* records,
                                 size_t record_offset, int n, int ntiles, hipStream_t st) {
  if (ntiles <= 0 || n <= 0) return hipErrorInvalidValue;
  int chunk = 1, nranges = 1;
  fold_ranges(ntiles, &chunk, &nranges);
  hipLaunchKernelGGL(fold_tiles_many_kernel<NSTAT>, dim3(nranges, n), dim3(1024), 0, st,
                     partials, ntiles, chunk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gather_folds_many_kernel<NSTAT>, dim3(1, n), dim3(SumShape<NSTAT>::VP), 0,
                     st, partials, nranges, chunk, records, record_offset);
  return hipGetLastError();
}

// out[NSTAT] = sum of the partials over all tiles (partials unchanged).
template <int NSTAT>
hipError_t open_sums(const double* partials, int ntiles, double* out, hipStream_t st) {
  if (ntiles <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(open_sums_kernel<NSTAT>, dim3(1), dim3(1024), 0, st, partials, ntiles, out);
  return hipGetLastError();
}

}  // namespace flb
