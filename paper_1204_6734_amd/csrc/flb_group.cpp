// flb_group.cpp — lattices and ensembles.  Both are a "group" of slots that
// share a stream, a device clock and one batched step launch per step; a
// lattice is a group of one slot (and is the only kind with the
// structure-factor pipeline).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
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

static size_t storage_size(int storage) { return storage == 0 ? sizeof(double) : sizeof(float); }

// Lay out every device array of the group in `a` (a.base may be null to
// size it).
void Group::layout(Arena& a) {
  const int n = (int)P.size();
  d_slots = a.take<SlotDesc>(n);
  d_prefix = a.take<int>(n + 2);
  d_clock = a.take<uint64_t>(1);
  d_err = a.take<int>(n);
  d_err_step = a.take<unsigned long long>(n);
  d_open = a.take<double>(kNStat);
  d_B = a.take<double>(81);
  d_mode = a.take<double2>(kModeBlocks);
  d_close = a.take<double*>(2 * (size_t)n);
  pop.resize(n);
  d_partials.assign(n, nullptr);
  d_records.assign(n, nullptr);
  size_t max_sites = 0;
  for (int s = 0; s < n; ++s) {
    const size_t N = (size_t)P[s].nx * P[s].ny;
    max_sites = std::max(max_sites, N);
    pop[s] = a.take<char>(population_elems(P[s].nx, P[s].ny) * storage_size(storage));
    if (P[s].sample_every > 0) {
      d_partials[s] = a.take<double>((size_t)hdesc[s].ntiles * kNStat);
      d_records[s] = a.take<double>((size_t)kMaxTimeBlocks * kNStat);
    }
  }
  // staging for host I/O, one band of rows at a time
  int maxnx = 0, maxny = 0;
  for (auto& p : P) {
    maxnx = std::max(maxnx, p.nx);
    maxny = std::max(maxny, p.ny);
  }
  band_rows = std::max(1, std::min(maxny, (int)((1u << 22) / (unsigned)maxnx)));
  d_io = a.take<double>((size_t)9 * band_rows * maxnx);
  if (n == 1 && P[0].sk_every > 0) {
    const size_t N = max_sites, cplx = 2 * storage_size(storage);
    d_z = a.take<char>(2 * N * cplx);
    d_zt = a.take<char>(2 * N * cplx);
    d_skacc = a.take<double>(5 * sk_half());
    d_twx = a.take<char>(P[0].nx * cplx);
    d_twy = a.take<char>(P[0].ny * cplx);
  }
}

int Group::init(const flb_params* ps, int n, void* stream, void* dev_buf, size_t dev_bytes) {
  if (n <= 0) return set_error(FLB_E_ARG, "need at least one lattice");
  for (int s = 0; s < n; ++s) {
    const int rc = check_params(&ps[s]);
    if (rc != FLB_OK) return rc;
    if (ps[s].nx != ps[0].nx || ps[s].ny != ps[0].ny || ps[s].precision != ps[0].precision ||
        ps[s].basis != ps[0].basis)
      return set_error(FLB_E_ARG, "ensemble members must share nx, ny, precision and basis");
    if (n > 1 && ps[s].sk_every > 0)
      return set_error(FLB_E_ARG, "structure factors are available for single lattices only");
  }
  P.assign(ps, ps + n);
  storage = ps[0].precision == FLB_FP64 ? 0 : 1;
  basis = ps[0].basis;
  compute = 1;
  for (int s = 0; s < n; ++s) compute = std::min(compute, compute_precision(&ps[s]));
  // launch classes: FP32-compute members first, then FP64-compute members
  corder.clear();
  nclass = 0;
  for (int cc : {1, 0}) {
    const int first = (int)corder.size();
    for (int s = 0; s < n; ++s)
      if (compute_precision(&ps[s]) == cc) corder.push_back(s);
    if ((int)corder.size() > first) {
      ccompute[nclass] = cc;
      cfirst[nclass] = first;
      ccount[nclass] = (int)corder.size() - first;
      ++nclass;
    }
  }
  hdesc.assign(n, SlotDesc{});
  prefix.assign(n + 1, 0);
  for (int s = 0; s < n; ++s) {
    fill_slot(&ps[s], &hdesc[s]);
    prefix[s + 1] = prefix[s] + hdesc[s].ntiles;
  }
  total_tiles = prefix[n];
  Arena sizing;
  layout(sizing);
  need_bytes = sizing.used + 256;
  if (dev_buf) {
    if (dev_bytes < need_bytes)
      return set_error(FLB_E_ARG, "device buffer too small: %zu < %zu bytes", dev_bytes,
                       need_bytes);
    dev = dev_buf;
    own_mem = false;
  } else {
    hipError_t e = hipMalloc(&dev, need_bytes);
    if (e != hipSuccess) {
      dev = nullptr;
      return set_error(FLB_E_OOM, "hipMalloc(%zu): %s", need_bytes, hipGetErrorString(e));
    }
    own_mem = true;
  }
  Arena a;
  a.base = (char*)(((uintptr_t)dev + 255) & ~(uintptr_t)255);
  layout(a);
  if (stream) {
    st = (hipStream_t)stream;
    own_stream = false;
  } else {
    HIPC(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    own_stream = true;
  }
  hipDeviceProp_t prop;
  int dev_id = 0;
  HIPC(hipGetDevice(&dev_id));
  HIPC(hipGetDeviceProperties(&prop, dev_id));
  max_lds = prop.sharedMemPerBlock;
  device = dev_id;
  if (d_skacc && (!sk_transform_supported(P[0].nx, storage, max_lds) ||
                  !sk_transform_supported(P[0].ny, storage, max_lds)))
    return set_error(FLB_E_ARG,
                     "structure factors need sides that are powers of two up to %d (FP64) or "
                     "%d (FP32) or at most %d",
                     (int)(max_lds / sizeof(double2)), (int)(max_lds / sizeof(float2)),
                     kMaxDirectDft);
  launch = tuned_launch(*this);
  // per-slot pointers and measurement bases
  mt0.assign(n, std::vector<double>(81));
  stats.assign(n, Stats{});
  for (int s = 0; s < n; ++s) {
    hdesc[s].pop = pop[s];
    hdesc[s].partials = d_partials[s];
    hdesc[s].skz = d_z;
    hdesc[s].err = d_err + s;
    hdesc[s].err_step = d_err_step + s;
    hdesc[s].t0 = 0;
    hdesc[s].tend = 0x7FFFFFFFFFFFFFFFull;  // never
    fnorm_rows(ps[s].ux0, ps[s].uy0, mt0[s].data());
    stats[s].reset(ps[s].block_steps);
  }
  {
    std::vector<SlotDesc> dev_desc(n);
    std::vector<int> dev_prefix;
    for (int c = 0; c < nclass; ++c) {
      int acc = 0;
      dev_prefix.push_back(0);
      for (int j = 0; j < ccount[c]; ++j) {
        const int s = corder[cfirst[c] + j];
        dev_desc[cfirst[c] + j] = hdesc[s];
        acc += hdesc[s].ntiles;
        dev_prefix.push_back(acc);
      }
      ctiles[c] = acc;
    }
    HIPC(hipMemcpy(d_slots, dev_desc.data(), n * sizeof(SlotDesc), hipMemcpyHostToDevice));
    std::vector<double*> close(2 * (size_t)n);
    for (int s = 0; s < n; ++s) {
      close[s] = d_partials[s];
      close[n + s] = d_records[s];
    }
    HIPC(hipMemcpy(d_close, close.data(), close.size() * sizeof(double*), hipMemcpyHostToDevice));
    HIPC(hipMemcpy(d_prefix, dev_prefix.data(), dev_prefix.size() * sizeof(int),
                   hipMemcpyHostToDevice));
  }
  HIPC(hipMemsetAsync(d_clock, 0, sizeof(uint64_t), st));
  HIPC(hipMemsetAsync(d_err, 0, n * sizeof(int), st));
  HIPC(hipMemsetAsync(d_err_step, 0xFF, n * sizeof(unsigned long long), st));
  for (int s = 0; s < n; ++s) {
    if (d_partials[s]) {
      HIPC(launch_fill(d_partials[s], (size_t)hdesc[s].ntiles * kNStat, 0.0, st));
      HIPC(launch_fill(d_records[s], (size_t)kMaxTimeBlocks * kNStat, 0.0, st));
    }
  }
  if (d_skacc) {
    const int nx = P[0].nx, ny = P[0].ny;
    HIPC(launch_fill(d_skacc, 5 * sk_half(), 0.0, st));
    // twiddles exp(-2 pi i k / n), k < n, in the storage precision
    for (int dim = 0; dim < 2; ++dim) {
      const int m = dim == 0 ? nx : ny;
      std::vector<double> tw(2 * (size_t)m);
      std::vector<float> twf(2 * (size_t)m);
      for (int k = 0; k < m; ++k) {
        const double ph = -2.0 * M_PI * (double)k / (double)m;
        tw[2 * k] = std::cos(ph);
        tw[2 * k + 1] = std::sin(ph);
        twf[2 * k] = (float)tw[2 * k];
        twf[2 * k + 1] = (float)tw[2 * k + 1];
      }
      const void* src = storage == 0 ? (const void*)tw.data() : (const void*)twf.data();
      HIPC(hipMemcpy(dim == 0 ? d_twx : d_twy, src, 2 * (size_t)m * storage_size(storage),
                     hipMemcpyHostToDevice));
    }
    HIPC(sk_prepare(max_lds));
  }
  for (int s = 0; s < n; ++s) {
    const flb_params& p = P[s];
    const double mu = p.init == FLB_INIT_THERMAL ? 3.0 * p.kT : 0.0;
    for (int y0 = 0; y0 < p.ny; y0 += band_rows) {
      const int rows = std::min(band_rows, p.ny - y0);
      HIPC(launch_init(storage, pop[s], hdesc[s].pitch, nullptr, nullptr, nullptr, p.rho0, p.ux0, p.uy0,
                       slot_shift(hdesc[s]), p.nx, p.ny, mu, hdesc[s].k0, hdesc[s].k1, 0, y0, rows,
                       st));
    }
  }
  t = 0;
  HIPC(hipStreamSynchronize(st));
  return FLB_OK;
}

Group::~Group() {
  if (st) (void)hipStreamSynchronize(st);
  for (auto& e : events) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (own_mem && dev) (void)hipFree(dev);
  if (own_stream && st) (void)hipStreamDestroy(st);
}

bool Group::sample_due(int s, uint64_t tt) const {
  const flb_params& p = P[s];
  return p.sample_every > 0 && tt % (uint64_t)p.sample_every == 0;
}

bool Group::sk_due(int s, uint64_t tt) const {
  const flb_params& p = P[s];
  return d_skacc && p.sk_every > 0 && tt % (uint64_t)p.sk_every == 0;
}

// Whether every slot closes a time block after the sample of time tt, all
// at the same record index, with no record merge first and one tile count:
// an ensemble whose replicas sample alike.  Then one batched launch closes
// them all, each with the additions of its own close.
bool Group::lockstep_close(uint64_t tt) const {
  const int n = (int)P.size();
  if (n < 2) return false;
  for (int s = 0; s < n; ++s)
    if (!sample_due(s, tt) || !stats[s].plain_close_next() || stats[s].nb != stats[0].nb ||
        hdesc[s].ntiles != hdesc[0].ntiles)
      return false;
  return true;
}

// Work after the step kernel of time tt: structure-factor transform and
// time-block bookkeeping.  After a graph replay the transforms of the
// chunk's steps ran inside the graph (replayed = true): only the counts and
// the time-block closes remain.
int Group::after_step(uint64_t tt, bool replayed) {
  const int n = (int)P.size();
  for (int s = 0; s < n; ++s) {
    if (sk_due(s, tt)) {
      if (!replayed)
        HIPC(launch_sk_sample(storage, d_z, d_zt, d_skacc, P[s].nx, P[s].ny, d_twx, d_twy,
                              max_lds, st));
      nsk += 1;
    }
  }
  if (lockstep_close(tt)) {
    uint64_t b = 0;
    for (int s = 0; s < n; ++s) b = stats[s].close_counted((uint64_t)P[s].nx * P[s].ny);
    HIPC(launch_close_block_many(d_close, d_close + n, (size_t)b * kNStat, n, hdesc[0].ntiles,
                                 st));
    return FLB_OK;
  }
  for (int s = 0; s < n; ++s)
    if (sample_due(s, tt))
      HIPC(stats[s].after_sample((uint64_t)P[s].nx * P[s].ny, d_partials[s], hdesc[s].ntiles,
                                 d_records[s], st));
  return FLB_OK;
}

// The step launches of one step: one per compute class.
hipError_t Group::launch_classes(uint32_t k, bool sample, int odd, LaunchCfg c) {
  for (int i = 0; i < nclass; ++i) {
    const hipError_t e = launch_step(storage, ccompute[i], basis, sample, odd, d_slots + cfirst[i],
                                     d_prefix + cfirst[i] + i, ccount[i], ctiles[i], d_clock, k,
                                     c, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

int Group::launch_one(uint32_t k, bool sample, int odd) {
  if (profiling) {
    std::pair<hipEvent_t, hipEvent_t> ev;
    HIPC(hipEventCreate(&ev.first));
    HIPC(hipEventCreate(&ev.second));
    HIPC(hipEventRecord(ev.first, st));
    HIPC(launch_classes(k, sample, odd, launch));
    HIPC(hipEventRecord(ev.second, st));
    events.push_back(ev);
    prof_launches += 1;
    return FLB_OK;
  }
  HIPC(launch_classes(k, sample, odd, launch));
  return FLB_OK;
}

// A captured chunk of graph_chunk steps can be replayed at every time that
// is a multiple of graph_chunk when each slot's sampling and structure-factor
// intervals divide the chunk: the pattern of sampled steps inside a chunk is
// then the same every time.
bool Group::graph_friendly() const {
  if (graph_chunk <= 0) return false;
  for (auto& p : P) {
    if (p.sample_every > 0 && graph_chunk % p.sample_every != 0) return false;
    if (d_skacc && p.sk_every > 0 && graph_chunk % p.sk_every != 0) return false;
  }
  return true;
}

// Steps from time t until (and including) the step whose sample closes a
// time block of some slot; replays must not straddle such a step.
uint64_t Group::steps_to_close() const {
  uint64_t m = ~0ull;
  for (int s = 0; s < (int)P.size(); ++s) {
    const uint64_t se = (uint64_t)P[s].sample_every;
    if (se == 0 || stats[s].tb_len == 0) continue;
    const uint64_t left = stats[s].tb_len - stats[s].tb_fill;  // samples to the close
    const uint64_t first = (t + se - 1) / se * se;              // next sampled time
    m = std::min(m, first + (left - 1) * se - t + 1);
  }
  return m;
}

int Group::capture_graph() {
  if (graph_exec) return FLB_OK;
  HIPC(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  for (int k = 0; k < graph_chunk; ++k) {
    // replays start at multiples of graph_chunk (even), so step k of a chunk
    // has parity k & 1 and a slot samples there iff k is a multiple of its
    // interval; a structure-factor step also takes the sampling variant (it
    // writes the fields) and is followed by its transform
    bool sample = false;
    for (int s = 0; s < (int)P.size(); ++s)
      sample |= sample_due(s, (uint64_t)k) || sk_due(s, (uint64_t)k);
    hipError_t e = launch_classes((uint32_t)k, sample, k & 1, launch);
    for (int s = 0; s < (int)P.size() && e == hipSuccess; ++s)
      if (sk_due(s, (uint64_t)k))
        e = launch_sk_sample(storage, d_z, d_zt, d_skacc, P[s].nx, P[s].ny, d_twx, d_twy,
                             max_lds, st);
    if (e != hipSuccess) {
      hipGraph_t g;
      (void)hipStreamEndCapture(st, &g);
      if (g) (void)hipGraphDestroy(g);
      return hip_fail(e, "capture step");
    }
  }
  HIPC(launch_tick(d_clock, (uint64_t)graph_chunk, st));
  HIPC(hipStreamEndCapture(st, &graph));
  HIPC(hipGraphInstantiate(&graph_exec, graph, nullptr, nullptr, 0));
  return FLB_OK;
}

int Group::step(uint64_t nsteps) {
  const int n = (int)P.size();
  const uint64_t K = (uint64_t)graph_chunk;
  const bool use_graph = graph_friendly();
  uint64_t done = 0;
  while (done < nsteps) {
    const uint64_t left = nsteps - done;
    if (use_graph && left >= K && t % K == 0 && steps_to_close() >= K) {
      int rc = capture_graph();
      if (rc != FLB_OK) return rc;
      if (profiling) {
        std::pair<hipEvent_t, hipEvent_t> ev;
        HIPC(hipEventCreate(&ev.first));
        HIPC(hipEventCreate(&ev.second));
        HIPC(hipEventRecord(ev.first, st));
        HIPC(hipGraphLaunch(graph_exec, st));
        HIPC(hipEventRecord(ev.second, st));
        events.push_back(ev);
        prof_launches += K;
      } else {
        HIPC(hipGraphLaunch(graph_exec, st));
      }
      for (uint64_t k = 0; k < K; ++k) {
        rc = after_step(t + k, true);
        if (rc != FLB_OK) return rc;
      }
      t += K;
      done += K;
      continue;
    }
    // eager chunk: up to 2^30 steps; with graphs, only up to the next
    // multiple of the chunk length or the next time-block close, after which
    // replays can resume
    uint64_t chunk = std::min<uint64_t>(left, 1ull << 30);
    if (use_graph) {
      const uint64_t to_align = t % K == 0 ? K : K - t % K;
      chunk = std::min(chunk, std::min(to_align, std::max<uint64_t>(1, steps_to_close())));
    }
    for (uint64_t k = 0; k < chunk; ++k) {
      const uint64_t tt = t + k;
      bool sample = false;
      for (int s = 0; s < n; ++s) sample |= sample_due(s, tt) || sk_due(s, tt);
      int rc = launch_one((uint32_t)k, sample, (int)(tt & 1));
      if (rc != FLB_OK) return rc;
      rc = after_step(tt);
      if (rc != FLB_OK) return rc;
    }
    HIPC(launch_tick(d_clock, chunk, st));
    t += chunk;
    done += chunk;
  }
  return FLB_OK;
}

int Group::sync() {
  HIPC(hipStreamSynchronize(st));
  const int n = (int)P.size();
  std::vector<int> err(n);
  std::vector<unsigned long long> es(n);
  HIPC(hipMemcpy(err.data(), d_err, n * sizeof(int), hipMemcpyDeviceToHost));
  HIPC(hipMemcpy(es.data(), d_err_step, n * sizeof(unsigned long long), hipMemcpyDeviceToHost));
  int code = FLB_OK;
  for (int s = 0; s < n; ++s) {
    err_step_host = -1;
    if (err[s]) {
      // own time of slot s at the failing step
      const int64_t stp = (int64_t)es[s];
      if (err[s] & kErrInvalidVelocity) {
        code = set_error(FLB_E_INVALID_VELOCITY,
                         "lattice %d: local velocity outside the validity region at step %lld",
                         s, (long long)stp);
      } else {
        code = set_error(FLB_E_NONFINITE, "lattice %d: non-finite state at step %lld", s,
                         (long long)stp);
      }
      err_step_host = stp;
      return code;
    }
  }
  return code;
}

int Group::read_populations(int s, double* f) {
  return read_rows(s, 0, P[s].ny, f);
}

// Rows [y0, y0 + nrows) of slot s, unshifted FP64, [9][nrows][nx].
int Group::read_rows(int s, int y0, int nrows, double* f) {
  int rc = sync();
  if (rc != FLB_OK) return rc;
  const flb_params& p = P[s];
  if (y0 < 0 || nrows < 0 || y0 + nrows > p.ny)
    return set_error(FLB_E_ARG, "rows [%d, %d) outside 0..%d", y0, y0 + nrows, p.ny);
  const size_t N = (size_t)p.nx * nrows;
  for (int b0 = y0; b0 < y0 + nrows; b0 += band_rows) {
    const int rows = std::min(band_rows, y0 + nrows - b0);
    HIPC(launch_read_state(storage, pop[s], hdesc[s].pitch, d_io, p.nx, p.ny, (int)(t & 1), slot_shift(hdesc[s]),
                           b0, rows, st));
    const size_t B = (size_t)rows * p.nx;
    for (int i = 0; i < 9; ++i)
      HIPC(hipMemcpyAsync(f + i * N + (size_t)(b0 - y0) * p.nx, d_io + i * B, B * sizeof(double),
                          hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
  }
  return FLB_OK;
}

int Group::set_populations(int s, const double* f, uint64_t tnew) {
  HIPC(hipStreamSynchronize(st));
  const flb_params& p = P[s];
  const size_t N = (size_t)p.nx * p.ny;
  if (P.size() != 1) return set_error(FLB_E_STATE, "set_populations needs a single lattice");
  t = tnew;
  HIPC(hipMemcpyAsync(d_clock, &t, sizeof(uint64_t), hipMemcpyHostToDevice, st));
  for (int y0 = 0; y0 < p.ny; y0 += band_rows) {
    const int rows = std::min(band_rows, p.ny - y0);
    const size_t B = (size_t)rows * p.nx;
    for (int i = 0; i < 9; ++i)
      HIPC(hipMemcpyAsync(d_io + i * B, f + i * N + (size_t)y0 * p.nx, B * sizeof(double),
                          hipMemcpyHostToDevice, st));
    HIPC(launch_write_state(storage, pop[s], hdesc[s].pitch, d_io, p.nx, p.ny, (int)(t & 1), slot_shift(hdesc[s]),
                            y0, rows, st));
    HIPC(hipStreamSynchronize(st));
  }
  return FLB_OK;
}

int Group::set_fields(int s, const double* rho, const double* ux, const double* uy) {
  HIPC(hipStreamSynchronize(st));
  const flb_params& p = P[s];
  for (int y0 = 0; y0 < p.ny; y0 += band_rows) {
    const int rows = std::min(band_rows, p.ny - y0);
    const size_t B = (size_t)rows * p.nx, off = (size_t)y0 * p.nx;
    HIPC(hipMemcpyAsync(d_io, rho + off, B * sizeof(double), hipMemcpyHostToDevice, st));
    HIPC(hipMemcpyAsync(d_io + B, ux + off, B * sizeof(double), hipMemcpyHostToDevice, st));
    HIPC(hipMemcpyAsync(d_io + 2 * B, uy + off, B * sizeof(double), hipMemcpyHostToDevice, st));
    HIPC(launch_init(storage, pop[s], hdesc[s].pitch, d_io, d_io + B, d_io + 2 * B, p.rho0, p.ux0, p.uy0,
                     slot_shift(hdesc[s]), p.nx, p.ny, 0.0, hdesc[s].k0, hdesc[s].k1,
                     (int)(t & 1), y0, rows, st));
    HIPC(hipStreamSynchronize(st));
  }
  return FLB_OK;
}

int Group::read_moments(int s, int at, double* m) {
  int rc = sync();
  if (rc != FLB_OK) return rc;
  const flb_params& p = P[s];
  const size_t N = (size_t)p.nx * p.ny;
  const double* B = nullptr;
  if (at == FLB_AT_U0 || at == FLB_AT_HERMITE) {
    double h[81];
    if (at == FLB_AT_U0) std::memcpy(h, mt0[s].data(), sizeof(h));
    else hermite_rows(h);
    HIPC(hipMemcpyAsync(d_B, h, sizeof(h), hipMemcpyHostToDevice, st));
    HIPC(hipStreamSynchronize(st));
    B = d_B;
  } else if (at != FLB_AT_LOCAL) {
    return set_error(FLB_E_ARG, "unknown moment basis %d", at);
  }
  for (int y0 = 0; y0 < p.ny; y0 += band_rows) {
    const int rows = std::min(band_rows, p.ny - y0);
    HIPC(launch_moments(storage, pop[s], hdesc[s].pitch, B, d_io, p.nx, p.ny, (int)(t & 1), p.rho0, p.ux0,
                        p.uy0, slot_shift(hdesc[s]), d_err + s, y0, rows, st));
    const size_t Bn = (size_t)rows * p.nx;
    for (int a = 0; a < 9; ++a)
      HIPC(hipMemcpyAsync(m + a * N + (size_t)y0 * p.nx, d_io + a * Bn, Bn * sizeof(double),
                          hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
  }
  return sync();
}

int Group::read_covariance(int s, flb_cov* out) {
  int rc = sync();
  if (rc != FLB_OK) return rc;
  const flb_params& p = P[s];
  std::vector<double> rec;
  double open[kNStat] = {0};
  if (d_partials[s]) {
    HIPC(launch_open_sum(d_partials[s], hdesc[s].ntiles, d_open, st));
    HIPC(hipMemcpyAsync(open, d_open, sizeof(open), hipMemcpyDeviceToHost, st));
    rec.resize((size_t)std::max<uint64_t>(stats[s].nb, 1) * kNStat);
    if (stats[s].nb > 0)
      HIPC(hipMemcpyAsync(rec.data(), d_records[s], stats[s].nb * kNStat * sizeof(double),
                          hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
  }
  return finish_covariance(stats[s], rec, open, (uint64_t)p.nx * p.ny, mt0[s].data(), out);
}

int Group::reset_stats() {
  HIPC(hipStreamSynchronize(st));
  for (int s = 0; s < (int)P.size(); ++s) {
    stats[s].reset(P[s].block_steps);
    if (d_partials[s]) {
      HIPC(launch_fill(d_partials[s], (size_t)hdesc[s].ntiles * kNStat, 0.0, st));
      HIPC(launch_fill(d_records[s], (size_t)kMaxTimeBlocks * kNStat, 0.0, st));
    }
  }
  if (d_skacc) HIPC(launch_fill(d_skacc, 5 * sk_half(), 0.0, st));
  nsk = 0;
  HIPC(hipStreamSynchronize(st));
  return FLB_OK;
}

int Group::read_structure_factor(int which, double* out) {
  int rc = sync();
  if (rc != FLB_OK) return rc;
  if (!d_skacc) return set_error(FLB_E_STATE, "structure factors are off (sk_every = 0)");
  if (which < 0 || which > 4) return set_error(FLB_E_ARG, "unknown structure factor %d", which);
  const int nx = P[0].nx, ny = P[0].ny;
  const size_t H = sk_half();
  std::vector<double> tmp(H);  // device order [kx][ky], kx <= nx/2
  HIPC(hipMemcpy(tmp.data(), d_skacc + which * H, H * sizeof(double), hipMemcpyDeviceToHost));
  const double norm = nsk > 0 ? 1.0 / ((double)nsk * (double)nx * (double)ny) : 0.0;
  for (int kx = 0; kx < nx; ++kx)
    for (int ky = 0; ky < ny; ++ky) {
      double v;
      if (kx <= nx / 2) {
        v = tmp[(size_t)kx * ny + ky];
      } else {  // the value at -k: equal, or the conjugate for the cross term
        v = tmp[(size_t)(nx - kx) * ny + (ky == 0 ? 0 : ny - ky)];
        if (which == FLB_SK_JXJY_IM) v = -v;
      }
      out[(size_t)ky * nx + kx] = v * norm;
    }
  return FLB_OK;
}

int Group::read_fourier_mode(int which, int kx, int ky, double out[2]) {
  int rc = sync();
  if (rc != FLB_OK) return rc;
  if (which < 0 || which > 2) return set_error(FLB_E_ARG, "unknown field %d", which);
  const flb_params& p = P[0];
  const int nkx = ((kx % p.nx) + p.nx) % p.nx, nky = ((ky % p.ny) + p.ny) % p.ny;
  int gx, gy;
  const int nblocks = fourier_mode_grid(p.nx, p.ny, kModeBlocks, &gx, &gy);
  HIPC(launch_fourier_mode(storage, pop[0], hdesc[0].pitch, d_mode, kModeBlocks, p.nx, p.ny,
                           (int)(t & 1), which, nkx, nky, p.ux0, p.uy0, st));
  std::vector<double2> part(nblocks);
  HIPC(hipMemcpyAsync(part.data(), d_mode, nblocks * sizeof(double2), hipMemcpyDeviceToHost,
                      st));
  HIPC(hipStreamSynchronize(st));
  double sr = 0, si = 0;
  for (auto& v : part) {
    sr += v.x;
    si += v.y;
  }
  out[0] = sr;
  out[1] = si;
  return FLB_OK;
}

// Checkpoint layout: header, then the nine storage planes in natural order.
struct CkptHeader {
  char magic[8];
  uint64_t t;
  flb_params p;
  uint64_t payload;
};

size_t Group::checkpoint_bytes() const {
  return sizeof(CkptHeader) + 9 * (size_t)P[0].nx * P[0].ny * storage_size(storage);
}

int Group::checkpoint(void* host, size_t bytes) {
  int rc = sync();
  if (rc != FLB_OK) return rc;
  if (bytes < checkpoint_bytes()) return set_error(FLB_E_ARG, "checkpoint buffer too small");
  CkptHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, "FLBCKPT1", 8);
  h.t = t;
  h.p = P[0];
  h.payload = checkpoint_bytes() - sizeof(CkptHeader);
  std::memcpy(host, &h, sizeof(h));
  char* dst = (char*)host + sizeof(h);
  const flb_params& p = P[0];
  const size_t N = (size_t)p.nx * p.ny, es = storage_size(storage);
  for (int y0 = 0; y0 < p.ny; y0 += band_rows) {
    const int rows = std::min(band_rows, p.ny - y0);
    const size_t B = (size_t)rows * p.nx;
    HIPC(launch_raw_state(storage, pop[0], hdesc[0].pitch, d_io, p.nx, p.ny, (int)(t & 1), 1, y0, rows, st));
    for (int i = 0; i < 9; ++i)
      HIPC(hipMemcpyAsync(dst + (i * N + (size_t)y0 * p.nx) * es, (char*)d_io + i * B * es, B * es,
                          hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
  }
  return FLB_OK;
}

int Group::restore(const void* host, size_t bytes) {
  HIPC(hipStreamSynchronize(st));
  if (bytes < sizeof(CkptHeader)) return set_error(FLB_E_ARG, "checkpoint too short");
  CkptHeader h;
  std::memcpy(&h, host, sizeof(h));
  if (std::memcmp(h.magic, "FLBCKPT1", 8) != 0) return set_error(FLB_E_ARG, "not a checkpoint");
  const flb_params& p = P[0];
  if (h.p.nx != p.nx || h.p.ny != p.ny || h.p.precision != p.precision ||
      h.payload + sizeof(h) != checkpoint_bytes() || bytes < checkpoint_bytes())
    return set_error(FLB_E_ARG, "checkpoint does not match this lattice");
  // the stored values are offsets from f^0(rho0, u0): the reference state must agree
  if (h.p.rho0 != p.rho0 || h.p.ux0 != p.ux0 || h.p.uy0 != p.uy0)
    return set_error(FLB_E_ARG, "checkpoint taken with another rho0 or u0");
  t = h.t;
  HIPC(hipMemcpyAsync(d_clock, &t, sizeof(uint64_t), hipMemcpyHostToDevice, st));
  const char* src = (const char*)host + sizeof(h);
  const size_t N = (size_t)p.nx * p.ny, es = storage_size(storage);
  for (int y0 = 0; y0 < p.ny; y0 += band_rows) {
    const int rows = std::min(band_rows, p.ny - y0);
    const size_t B = (size_t)rows * p.nx;
    for (int i = 0; i < 9; ++i)
      HIPC(hipMemcpyAsync((char*)d_io + i * B * es, src + (i * N + (size_t)y0 * p.nx) * es, B * es,
                          hipMemcpyHostToDevice, st));
    HIPC(launch_raw_state(storage, pop[0], hdesc[0].pitch, d_io, p.nx, p.ny, (int)(t & 1), 0, y0, rows, st));
    HIPC(hipStreamSynchronize(st));
  }
  return reset_stats();
}

int Group::kernel_time(double* ms, uint64_t* launches) {
  HIPC(hipStreamSynchronize(st));
  double tot = 0;
  for (auto& e : events) {
    float m = 0;
    HIPC(hipEventElapsedTime(&m, e.first, e.second));
    tot += m;
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  events.clear();
  prof_ms += tot;
  if (ms) *ms = prof_ms;
  if (launches) *launches = prof_launches;
  prof_ms = 0;
  prof_launches = 0;
  return FLB_OK;
}

}  // namespace flb

// ===================================================================== C ABI
using flb::Group;

struct flb_lattice {
  Group g;
};
struct flb_ensemble {
  Group g;
};

extern "C" {

const char* flb_last_error(void);

size_t flb_lattice_bytes(const flb_params* p) {
  if (flb::check_params(p) != FLB_OK) return 0;
  Group g;
  g.P.assign(p, p + 1);
  g.storage = p->precision == FLB_FP64 ? 0 : 1;
  g.hdesc.assign(1, flb::SlotDesc{});
  flb::fill_slot(p, &g.hdesc[0]);
  flb::Arena a;
  g.layout(a);
  return a.used + 256;
}

static int lattice_make(const flb_params* p, void* stream, void* buf, size_t bytes,
                        flb_lattice** out) {
  if (!out) return flb::set_error(FLB_E_ARG, "null output handle");
  *out = nullptr;
  flb_lattice* L = new (std::nothrow) flb_lattice();
  if (!L) return flb::set_error(FLB_E_OOM, "host allocation");
  const int rc = L->g.init(p, 1, stream, buf, bytes);
  if (rc != FLB_OK) {
    delete L;
    return rc;
  }
  *out = L;
  return FLB_OK;
}

int flb_lattice_create(const flb_params* p, void* hip_stream, flb_lattice** out) {
  return lattice_make(p, hip_stream, nullptr, 0, out);
}

int flb_lattice_create_on(const flb_params* p, void* dev_buf, size_t bytes, void* hip_stream,
                          flb_lattice** out) {
  if (!dev_buf) return flb::set_error(FLB_E_ARG, "null device buffer");
  return lattice_make(p, hip_stream, dev_buf, bytes, out);
}

#define NEED(h) \
  if (!(h)) return flb::set_error(FLB_E_ARG, "null handle")

int flb_lattice_set_fields(flb_lattice* L, const double* rho, const double* ux, const double* uy) {
  NEED(L);
  if (!rho || !ux || !uy) return flb::set_error(FLB_E_ARG, "null field");
  return L->g.set_fields(0, rho, ux, uy);
}
int flb_lattice_set_populations(flb_lattice* L, const double* f, uint64_t t) {
  NEED(L);
  if (!f) return flb::set_error(FLB_E_ARG, "null populations");
  return L->g.set_populations(0, f, t);
}
int flb_lattice_set_graph_chunk(flb_lattice* L, int32_t steps) {
  NEED(L);
  if (steps < 0 || steps > (1 << 16)) return flb::set_error(FLB_E_ARG, "bad chunk %d", steps);
  const hipError_t e = hipStreamSynchronize(L->g.st);  // no replay in flight
  if (e != hipSuccess) return flb::hip_fail(e, "sync");
  L->g.drop_graph();
  L->g.graph_chunk = steps + (steps & 1);  // even: replays keep the streaming phase
  return FLB_OK;
}
int flb_lattice_step(flb_lattice* L, uint64_t n) {
  NEED(L);
  return L->g.step(n);
}
int flb_lattice_sync(flb_lattice* L) {
  NEED(L);
  return L->g.sync();
}
int flb_lattice_read_populations(flb_lattice* L, double* f) {
  NEED(L);
  if (!f) return flb::set_error(FLB_E_ARG, "null output");
  return L->g.read_populations(0, f);
}
int flb_lattice_read_rows(flb_lattice* L, int32_t y0, int32_t nrows, double* f) {
  NEED(L);
  if (!f) return flb::set_error(FLB_E_ARG, "null output");
  return L->g.read_rows(0, y0, nrows, f);
}
int flb_lattice_read_moments(flb_lattice* L, int32_t at, double* m) {
  NEED(L);
  if (!m) return flb::set_error(FLB_E_ARG, "null output");
  return L->g.read_moments(0, at, m);
}
int flb_lattice_read_covariance(flb_lattice* L, flb_cov* out) {
  NEED(L);
  if (!out) return flb::set_error(FLB_E_ARG, "null output");
  return L->g.read_covariance(0, out);
}
int flb_lattice_read_structure_factor(flb_lattice* L, int32_t which, double* out) {
  NEED(L);
  if (!out) return flb::set_error(FLB_E_ARG, "null output");
  return L->g.read_structure_factor(which, out);
}
int flb_lattice_read_fourier_mode(flb_lattice* L, int32_t which, int32_t kx, int32_t ky,
                                  double out[2]) {
  NEED(L);
  if (!out) return flb::set_error(FLB_E_ARG, "null output");
  return L->g.read_fourier_mode(which, kx, ky, out);
}
int flb_lattice_reset_stats(flb_lattice* L) {
  NEED(L);
  return L->g.reset_stats();
}
size_t flb_lattice_checkpoint_bytes(flb_lattice* L) { return L ? L->g.checkpoint_bytes() : 0; }
int flb_lattice_checkpoint(flb_lattice* L, void* host, size_t bytes) {
  NEED(L);
  if (!host) return flb::set_error(FLB_E_ARG, "null buffer");
  return L->g.checkpoint(host, bytes);
}
int flb_lattice_restore(flb_lattice* L, const void* host, size_t bytes) {
  NEED(L);
  if (!host) return flb::set_error(FLB_E_ARG, "null buffer");
  return L->g.restore(host, bytes);
}
int flb_lattice_population_buffer(flb_lattice* L, void** dev, size_t* bytes, uint64_t* t) {
  NEED(L);
  if (!dev || !bytes || !t) return flb::set_error(FLB_E_ARG, "null output");
  const hipError_t e = hipStreamSynchronize(L->g.st);
  if (e != hipSuccess) return flb::hip_fail(e, "sync");
  const flb_params& p = L->g.P[0];
  *dev = L->g.pop[0];
  *bytes = flb::population_elems(p.nx, p.ny) * (L->g.storage == 0 ? 8 : 4);
  *t = L->g.t;
  return FLB_OK;
}
uint64_t flb_lattice_time(flb_lattice* L) { return L ? L->g.t : 0; }
int64_t flb_lattice_error_step(flb_lattice* L) { return L ? L->g.err_step_host : -1; }
int flb_lattice_profile(flb_lattice* L, int32_t on) {
  NEED(L);
  L->g.profiling = on != 0;
  return FLB_OK;
}
int flb_lattice_kernel_time(flb_lattice* L, double* ms, uint64_t* launches) {
  NEED(L);
  return L->g.kernel_time(ms, launches);
}
void flb_lattice_destroy(flb_lattice* L) { delete L; }

int flb_ensemble_create(const flb_params* ps, int32_t n, void* hip_stream, flb_ensemble** out) {
  if (!out || !ps) return flb::set_error(FLB_E_ARG, "null argument");
  *out = nullptr;
  flb_ensemble* E = new (std::nothrow) flb_ensemble();
  if (!E) return flb::set_error(FLB_E_OOM, "host allocation");
  const int rc = E->g.init(ps, n, hip_stream, nullptr, 0);
  if (rc != FLB_OK) {
    delete E;
    return rc;
  }
  *out = E;
  return FLB_OK;
}
int flb_ensemble_set_graph_chunk(flb_ensemble* E, int32_t steps) {
  NEED(E);
  if (steps < 0 || steps > (1 << 16)) return flb::set_error(FLB_E_ARG, "bad chunk %d", steps);
  const hipError_t e = hipStreamSynchronize(E->g.st);  // no replay in flight
  if (e != hipSuccess) return flb::hip_fail(e, "sync");
  E->g.drop_graph();
  E->g.graph_chunk = steps + (steps & 1);  // even: replays keep the streaming phase
  return FLB_OK;
}
int flb_ensemble_step(flb_ensemble* E, uint64_t n) {
  NEED(E);
  return E->g.step(n);
}
int flb_ensemble_sync(flb_ensemble* E) {
  NEED(E);
  return E->g.sync();
}
int flb_ensemble_read_populations(flb_ensemble* E, int32_t i, double* f) {
  NEED(E);
  if (i < 0 || i >= (int)E->g.P.size() || !f) return flb::set_error(FLB_E_ARG, "bad replica");
  return E->g.read_populations(i, f);
}
int flb_ensemble_read_covariance(flb_ensemble* E, int32_t i, flb_cov* out) {
  NEED(E);
  if (i < 0 || i >= (int)E->g.P.size() || !out) return flb::set_error(FLB_E_ARG, "bad replica");
  return E->g.read_covariance(i, out);
}
int flb_ensemble_reset_stats(flb_ensemble* E) {
  NEED(E);
  return E->g.reset_stats();
}
uint64_t flb_ensemble_time(flb_ensemble* E) { return E ? E->g.t : 0; }
int flb_ensemble_profile(flb_ensemble* E, int32_t on) {
  NEED(E);
  E->g.profiling = on != 0;
  return FLB_OK;
}
int flb_ensemble_kernel_time(flb_ensemble* E, double* ms, uint64_t* launches) {
  NEED(E);
  return E->g.kernel_time(ms, launches);
}
void flb_ensemble_destroy(flb_ensemble* E) { delete E; }

int flb_lattice_autotune(flb_lattice* L, int32_t reps, flb_launch_config* results,
                         int32_t max_results, int32_t* n_results) {
  NEED(L);
  return L->g.autotune(reps, results, max_results, n_results);
}
int flb_ensemble_autotune(flb_ensemble* E, int32_t reps, flb_launch_config* results,
                          int32_t max_results, int32_t* n_results) {
  NEED(E);
  return E->g.autotune(reps, results, max_results, n_results);
}
int flb_lattice_set_launch(flb_lattice* L, const flb_launch_config* c) {
  NEED(L);
  return L->g.set_launch(c);
}
int flb_ensemble_set_launch(flb_ensemble* E, const flb_launch_config* c) {
  NEED(E);
  return E->g.set_launch(c);
}
int flb_lattice_get_launch(flb_lattice* L, flb_launch_config* c) {
  NEED(L);
  if (!c) return flb::set_error(FLB_E_ARG, "null output");
  *c = flb_launch_config{L->g.launch.tiles_per_block, L->g.launch.grid_blocks, 0.0};
  return FLB_OK;
}
int flb_ensemble_get_launch(flb_ensemble* E, flb_launch_config* c) {
  NEED(E);
  if (!c) return flb::set_error(FLB_E_ARG, "null output");
  *c = flb_launch_config{E->g.launch.tiles_per_block, E->g.launch.grid_blocks, 0.0};
  return FLB_OK;
}

}  // extern "C"
