// flb_noalloc.hip — flb_step_noalloc: the batched step (flb_step.hip) on
// populations held by the caller, with every intermediate (the slot
// descriptor, the tile prefix, the step clock, the error flags and the
// per-tile correlator partials) in one file-scope device array instead of
// memory the library allocates.  For callers that cannot allocate device
// memory: code under stream capture, serving loops that own their memory,
// harnesses that forbid it.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "flb.h"
#include "flb_kernels.hpp"
#include "flb_runtime.hpp"

namespace flb {
namespace {

// The descriptor block at the start of the scratch array; the per-tile
// partials follow at kPartialsOffset.
struct ScratchHead {
  SlotDesc slot;
  int prefix[2];
  int err;
  int pad_;
  unsigned long long err_step;
  uint64_t clock;
};
constexpr size_t kPartialsOffset = 4096;
static_assert(sizeof(ScratchHead) <= kPartialsOffset, "descriptor block fits");
constexpr size_t kScratchBytes =
    kPartialsOffset + (size_t)FLB_NOALLOC_MAX_TILES * kNStat * sizeof(double);
constexpr int kMaxDevices = 64;

// One per device, held by the code object for the life of the process.
// Host code never uses this name as an address: it uses the device address
// hipGetSymbolAddress returns (scratch_address below).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// The current device's address of `scratch`, looked up on the first call on
// that device (with the device current) and kept.
int scratch_address(char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return set_error(FLB_E_ARG, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return set_error(FLB_E_HIP, "hipGetSymbolAddress(scratch) returned null");
    g_scratch[dev] = p;
  }
  *out = static_cast<char*>(g_scratch[dev]);
  return FLB_OK;
}

// Writes the descriptor (passed by value), the tile prefix and the clock
// into the descriptor block and clears the error flags.
__global__ void noalloc_setup_kernel(ScratchHead* head, SlotDesc d, int ntiles) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  head->slot = d;
  head->prefix[0] = 0;
  head->prefix[1] = ntiles;
  head->err = 0;
  head->err_step = ~0ull;
  head->clock = 0;
}

// The call's outcome as an FLB_* code.
__global__ void noalloc_status_kernel(const ScratchHead* head, int32_t* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int e = head->err;
  *out = (e & kErrInvalidVelocity) ? FLB_E_INVALID_VELOCITY
                                   : ((e & kErrNonFinite) ? FLB_E_NONFINITE : FLB_OK);
}

}  // namespace
}  // namespace flb

extern "C" size_t flb_population_bytes(const flb_params* p) {
  if (flb::check_params(p) != FLB_OK) return 0;
  return flb::population_elems(p->nx, p->ny) * (p->precision == FLB_FP64 ? 8 : 4);
}

extern "C" int flb_step_noalloc(const flb_params* p, void* pop, uint64_t t0, uint64_t nsteps,
                                double* sums, int32_t* status, void* hip_stream) {
  using namespace flb;
  int rc = check_params(p);
  if (rc != FLB_OK) return rc;
  if (!pop) return set_error(FLB_E_ARG, "null populations");
  if (p->sk_every != 0)
    return set_error(FLB_E_ARG, "structure factors need library-owned buffers (sk_every = 0)");
  if (t0 >= (1ull << 62) || nsteps >= (1ull << 62))
    return set_error(FLB_E_ARG, "t0 and nsteps must be below 2^62");
  SlotDesc d;
  std::memset(&d, 0, sizeof(d));
  fill_slot(p, &d);
  const bool sampling = p->sample_every > 0;
  if (sampling && !sums) return set_error(FLB_E_ARG, "null sums with sample_every > 0");
  if (sampling && d.ntiles > FLB_NOALLOC_MAX_TILES)
    return set_error(FLB_E_ARG, "%d tiles of correlator partials exceed the scratch's %d",
                     d.ntiles, FLB_NOALLOC_MAX_TILES);
  char* base = nullptr;
  rc = scratch_address(&base);
  if (rc != FLB_OK) return rc;
  ScratchHead* head = reinterpret_cast<ScratchHead*>(base);
  double* partials = reinterpret_cast<double*>(base + kPartialsOffset);
  d.pop = pop;
  d.partials = sampling ? partials : nullptr;
  d.skz = nullptr;
  d.err = &head->err;
  d.err_step = &head->err_step;
  d.t0 = t0;
  d.tend = 0x7FFFFFFFFFFFFFFFull;
  const hipStream_t st = (hipStream_t)hip_stream;
  const int storage = p->precision == FLB_FP64 ? 0 : 1;
  const int compute = compute_precision(p);
  hipLaunchKernelGGL(noalloc_setup_kernel, dim3(1), dim3(64), 0, st, head, d, d.ntiles);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "noalloc set-up");
  if (sampling) {
    e = launch_fill(partials, (size_t)d.ntiles * kNStat, 0.0, st);
    if (e != hipSuccess) return hip_fail(e, "clear partials");
  }
  // steps in chunks whose index fits the kernels' 32-bit step offset; the
  // device clock advances after each chunk
  uint64_t done = 0;
  while (done < nsteps) {
    const uint64_t chunk = std::min<uint64_t>(nsteps - done, 1ull << 30);
    for (uint64_t k = 0; k < chunk; ++k) {
      const uint64_t t = t0 + done + k;
      const bool sample = sampling && t % (uint64_t)p->sample_every == 0;
      e = launch_step(storage, compute, p->basis, sample, (int)(t & 1), &head->slot, head->prefix,
                      1, d.ntiles, &head->clock, (uint32_t)k, LaunchCfg{}, st);
      if (e != hipSuccess) return hip_fail(e, "step");
    }
    e = launch_tick(&head->clock, chunk, st);
    if (e != hipSuccess) return hip_fail(e, "clock");
    done += chunk;
  }
  if (sampling) {
    e = launch_open_sum(partials, d.ntiles, sums, st);
    if (e != hipSuccess) return hip_fail(e, "sums");
  }
  if (status) {
    hipLaunchKernelGGL(noalloc_status_kernel, dim3(1), dim3(64), 0, st, head, status);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "status");
  }
  return FLB_OK;
}
