// flb_kernels.hpp — device-side data structures shared by the kernels and
// the host runtime of libflb (internal; not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace flb {

constexpr int kTileX = 64;   // sites of one wavefront: 64 consecutive sites of a row
constexpr int kTileY = 4;    // four wavefronts per 256-site tile
constexpr int kBlock = kTileX * kTileY;
constexpr int kWideTileMinNx = 256;  // rows this long use 256 x 1 tiles (else 64 x 4)
constexpr int kMaxTilesPerBlock = 4;  // workgroups of up to 1024 threads
constexpr int kMaxBlock = kBlock * kMaxTilesPerBlock;
constexpr int kNStat = 54;   // 9 first moments + 45 unique second moments
constexpr int kMaxTimeBlocks = 1024;
constexpr int kMaxDirectDft = 4096;  // longest row transformed by the O(n^2) DFT
enum : int { kErrInvalidVelocity = 1, kErrNonFinite = 2 };

// Population storage of one lattice (shifted values h = f - f^0(rho0, u0)):
// row-interleaved, the nine plane rows of lattice row y one after another,
// value i of site (x, y) at element (9 y + i) pitch + x, pitch = nx rounded
// up to a multiple of 64.  A wavefront's nine loads then fall into one
// 9 pitch stretch of memory instead of nine planes far apart (a copy with
// the step's access pattern ran 15 % faster this way than with planes).
//
// One lattice ("slot") as seen by the batched step kernel.  All slots of a
// launch share the storage and compute types and the basis variant.
struct SlotDesc {
  void* pop;            // storage, layout above
  double* partials;     // [ntiles][kNStat] open time-block sums (sampling)
  void* skz;            // [2][ny][nx] complex structure-factor planes (storage precision) or null
  int* err;             // error bits (atomicOr)
  unsigned long long* err_step;  // first failing step (atomicMin)
  int nx, ny, tiles_x, ntiles;
  uint32_t tx_magic, tx_shift;  // local tile t: row of tiles = (t * tx_magic) >> tx_shift
  uint32_t se_magic, se_shift;  // the same division by sample_every (when > 0)
  uint32_t sk_magic, sk_shift;  // and by sk_every (when > 0)
  uint64_t t0;          // own time = t0 + clock (mod 2^64)
  uint64_t tend;        // no update once own time >= tend (tend < 2^63)
  uint32_t k0, k1;      // Philox key = seed
  int sample_every;     // 0: never
  int sk_every;         // 0: never
  int noise;
  uint32_t pitch;       // elements per plane row (nx rounded up to kTileX)
  int wide;             // tile shape: 1 = 256 x 1 (four wavefronts along one row), 0 = 64 x 4
  int one_tau;          // all six relaxation times equal
  double rho0, ux0, uy0;
  double rt[6], xc[6];  // 1/tau, noise coefficients
  double xc2;           // mu (2 tau - 1) / tau^2 = xc^2 when one_tau
  double shift[9];      // f_i^0(rho0, u0): storage holds h = f - shift
  float rho0f, ux0f, uy0f, xc2f;  // single-precision copies
  float rtf[6], xcf[6], shiftf[9];
};

// Whether t is a multiple of m (m >= 1; magic, shift for m from magic_div):
// a multiply-shift for t < 2^31, the 64-bit remainder beyond.  Wave-uniform
// times keep this on the scalar unit, where the 64-bit remainder alone is a
// long instruction sequence.
__host__ __device__ __forceinline__ bool multiple_of(uint64_t t, uint32_t m, uint32_t magic,
                                                     uint32_t shift) {
  if ((t >> 31) == 0) {
    const uint32_t q = (uint32_t)(((uint64_t)(uint32_t)t * magic) >> shift);
    return (uint32_t)t == q * m;
  }
  return t % m == 0;
}

}  // namespace flb

namespace flb {
// Complex value of a real type.
template <typename T> struct Cplx;
template <> struct Cplx<double> { using type = double2; };
template <> struct Cplx<float> { using type = float2; };

// Launch shape of the batched step: tiles per workgroup (1, 2 or 4) and the
// grid (0: one workgroup per tile group; > 0, a multiple of 8: a persistent
// grid of that many workgroups striding over the tile groups).  Every shape
// computes bit-identical results.
struct LaunchCfg {
  int tiles_per_block = 1;
  int grid_blocks = 0;
};

// Nine FP64 values passed by value to utility kernels (the storage shift).
struct Shift9 {
  double v[9];
};
}  // namespace flb
