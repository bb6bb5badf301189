// flb_tune.cpp — launch-shape autotuner of the batched step.
//
// The step kernel can run with 1, 2 or 4 tiles of 64 x 4 sites per workgroup
// and with either one workgroup per tile group or a persistent grid that
// strides over the tile groups.  All shapes compute bit-identical results,
// so the choice is purely a matter of speed, which depends on the device,
// the precision and basis variant (register use, hence occupancy) and the
// number of tiles.  The tuner times each candidate on a copy of the real
// populations and keeps the fastest; choices are remembered per process.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "flb.h"
#include "flb_group.hpp"
#include "flb_runtime.hpp"

namespace flb {

#define HIPC(expr)                                    \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return hip_fail(e_, #expr); \
  } while (0)

namespace {

using Key = std::tuple<int, int, int, int, int>;  // device, storage, compute, basis, tiles

std::mutex g_cache_mu;
std::map<Key, LaunchCfg> g_cache;

Key key_of(const Group& g) {
  return Key{g.device, g.storage, g.compute, g.basis, g.total_tiles};
}

bool valid(const flb_launch_config& c) {
  return (c.tiles_per_block == 1 || c.tiles_per_block == 2 || c.tiles_per_block == 4) &&
         c.grid_blocks >= 0 && c.grid_blocks % 8 == 0;
}

// Candidate shapes: every tiles-per-workgroup choice with one workgroup per
// tile group, and persistent grids holding about 2, 4 or 6 wavefronts per
// SIMD (four SIMDs per CU) where that is fewer workgroups than tile groups.
std::vector<LaunchCfg> candidates(int total_tiles, int cus, int max_tpb) {
  std::vector<LaunchCfg> out;
  for (int tpb : {1, 2, 4}) {
    if (tpb > max_tpb) break;
    out.push_back(LaunchCfg{tpb, 0});
    const int ngroups = (total_tiles + tpb - 1) / tpb;
    for (int waves_per_simd : {2, 4, 6}) {
      // 4 tpb wavefronts per workgroup, 4 SIMDs per CU
      int blocks = cus * waves_per_simd / tpb;
      blocks = std::max(8, blocks / 8 * 8);
      if (blocks < ngroups) out.push_back(LaunchCfg{tpb, blocks});
    }
  }
  return out;
}

}  // namespace

LaunchCfg tuned_launch(const Group& g) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  auto it = g_cache.find(key_of(g));
  return it == g_cache.end() ? LaunchCfg{} : it->second;
}

void Group::drop_graph() {
  if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
  if (graph) (void)hipGraphDestroy(graph);
  graph_exec = nullptr;
  graph = nullptr;
}

int Group::set_launch(const flb_launch_config* c) {
  if (!c || !valid(*c))
    return set_error(FLB_E_ARG, "launch shape: tiles_per_block must be 1, 2 or 4 and "
                                "grid_blocks a non-negative multiple of 8");
  HIPC(hipStreamSynchronize(st));
  drop_graph();
  launch = LaunchCfg{c->tiles_per_block, c->grid_blocks};
  return FLB_OK;
}

int Group::autotune(int reps, flb_launch_config* results, int max_results, int* n_results) {
  if (reps < 1 || reps > 1000) return set_error(FLB_E_ARG, "reps must be in 1..1000");
  if (max_results < 0 || (max_results > 0 && !results))
    return set_error(FLB_E_ARG, "null results array");
  const int n = (int)P.size();
  HIPC(hipStreamSynchronize(st));
  int cus = 0;
  HIPC(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
  // snapshot of everything a trial step writes: populations and error flags
  std::vector<size_t> bytes(n);
  size_t total = 0;
  for (int s = 0; s < n; ++s) {
    bytes[s] = population_elems(P[s].nx, P[s].ny) * (storage == 0 ? sizeof(double) : sizeof(float));
    total += (bytes[s] + 255) & ~(size_t)255;
  }
  const size_t err_bytes = n * (sizeof(int) + sizeof(unsigned long long));
  char* snap = nullptr;
  hipError_t e = hipMalloc((void**)&snap, total + err_bytes);
  if (e != hipSuccess) return set_error(FLB_E_OOM, "autotune snapshot of %zu bytes", total);
  struct Free {
    char* p;
    ~Free() {
      if (p) (void)hipFree(p);
    }
  } free_snap{snap};
  auto copy = [&](bool save) -> hipError_t {
    size_t o = 0;
    for (int s = 0; s < n; ++s) {
      hipError_t r = save ? hipMemcpyAsync(snap + o, pop[s], bytes[s], hipMemcpyDeviceToDevice, st)
                          : hipMemcpyAsync(pop[s], snap + o, bytes[s], hipMemcpyDeviceToDevice, st);
      if (r != hipSuccess) return r;
      o += (bytes[s] + 255) & ~(size_t)255;
    }
    const size_t ei = n * sizeof(int);
    hipError_t r = save ? hipMemcpyAsync(snap + o, d_err, ei, hipMemcpyDeviceToDevice, st)
                        : hipMemcpyAsync(d_err, snap + o, ei, hipMemcpyDeviceToDevice, st);
    if (r != hipSuccess) return r;
    const size_t es = n * sizeof(unsigned long long);
    return save ? hipMemcpyAsync(snap + o + ei, d_err_step, es, hipMemcpyDeviceToDevice, st)
                : hipMemcpyAsync(d_err_step, snap + o + ei, es, hipMemcpyDeviceToDevice, st);
  };
  HIPC(copy(true));
  hipEvent_t e0, e1;
  HIPC(hipEventCreate(&e0));
  HIPC(hipEventCreate(&e1));
  struct Ev {
    hipEvent_t a, b;
    ~Ev() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } ev{e0, e1};
  // trial steps: the non-sampling kernel at the current time and parity
  // (steps k = 0, 1 of the device clock), so every pair returns the storage
  // to the phase it started in
  auto pair = [&](const LaunchCfg& c) -> hipError_t {
    for (uint32_t k = 0; k < 2; ++k) {
      hipError_t r = launch_classes(k, false, (int)((t + k) & 1), c);
      if (r != hipSuccess) return r;
    }
    return hipSuccess;
  };
  // FP64-compute step variants take at most two tiles per workgroup
  const std::vector<LaunchCfg> cand = candidates(total_tiles, cus, compute == 0 ? 2 : 4);
  std::vector<flb_launch_config> meas;
  for (const LaunchCfg& c : cand)
    meas.push_back(flb_launch_config{c.tiles_per_block, c.grid_blocks, 1e30});
  // warm the device up (clocks ramp over tens of milliseconds) for at least
  // 8 pairs or 50 ms, then time every candidate in two interleaved rounds and
  // keep each one's faster round.  The snapshot is put back whether or not
  // the trials succeed.
  auto trials = [&]() -> hipError_t {
    hipError_t r = hipEventRecord(e0, st);
    for (int w = 0; w < 1000 && r == hipSuccess; ++w) {
      r = pair(cand[0]);
      if (r == hipSuccess && w >= 7 && (w & 7) == 7) {
        r = hipEventRecord(e1, st);
        if (r == hipSuccess) r = hipEventSynchronize(e1);
        float ms = 0.f;
        if (r == hipSuccess) r = hipEventElapsedTime(&ms, e0, e1);
        if (r == hipSuccess && ms > 50.f) break;
      }
    }
    for (int round = 0; round < 2 && r == hipSuccess; ++round) {
      for (size_t i = 0; i < cand.size() && r == hipSuccess; ++i) {
        r = pair(cand[i]);  // first launches of a shape
        if (r == hipSuccess) r = hipEventRecord(e0, st);
        for (int k = 0; k < reps && r == hipSuccess; ++k) r = pair(cand[i]);
        if (r == hipSuccess) r = hipEventRecord(e1, st);
        if (r == hipSuccess) r = hipEventSynchronize(e1);
        float ms = 0.f;
        if (r == hipSuccess) r = hipEventElapsedTime(&ms, e0, e1);
        if (r == hipSuccess)
          meas[i].ms_per_step = std::min(meas[i].ms_per_step, ms / (2.0 * reps));
      }
    }
    return r;
  };
  const hipError_t tr = trials();
  const hipError_t back = copy(false);
  if (tr != hipSuccess) return hip_fail(tr, "autotune trial steps");
  if (back != hipSuccess) return hip_fail(back, "autotune: restoring the populations");
  HIPC(hipStreamSynchronize(st));
  std::stable_sort(meas.begin(), meas.end(),
                   [](const flb_launch_config& a, const flb_launch_config& b) {
                     return a.ms_per_step < b.ms_per_step;
                   });
  drop_graph();
  launch = LaunchCfg{meas[0].tiles_per_block, meas[0].grid_blocks};
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_cache[key_of(*this)] = launch;
  }
  for (int i = 0; i < std::min<int>(max_results, (int)meas.size()); ++i) results[i] = meas[i];
  if (n_results) *n_results = (int)meas.size();
  return FLB_OK;
}

}  // namespace flb
