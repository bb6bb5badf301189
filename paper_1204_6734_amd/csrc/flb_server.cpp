// flb_server.cpp — continuous batching of simulation requests.
//
// Requests wait in arrival order.  At every chunk boundary the scheduler
// retires finished requests (their correlators are read and their memory
// returned), then admits waiting requests in order while a slot is free and
// the head request's device footprint fits the memory budget (a first-fit
// arena carved from one allocation of the budget).  All admitted requests
// then advance together for `chunk_steps` steps: one batched step launch
// per step and compute precision covers every active lattice; a request that
// reaches its step count stops updating inside the chunk.  A request runs
// on its own clock (t = t0 + device clock), with noise keyed by its own
// seed, step and site and its correlator sums reduced per request in a
// fixed order, so its result does not depend on what else is in the batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "flb.h"
#include "flb_runtime.hpp"

namespace flb {

constexpr int kServerBlocks = 64;  // time-block records per request

#define HIPC(expr)                                    \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return hip_fail(e_, #expr); \
  } while (0)

// First-fit allocator over [0, cap).
struct FreeList {
  std::map<size_t, size_t> free;  // offset -> size
  size_t cap = 0, used = 0;
  void reset(size_t c) {
    cap = c;
    used = 0;
    free.clear();
    free[0] = c;
  }
  bool alloc(size_t n, size_t* off) {
    n = (n + 255) & ~(size_t)255;
    for (auto it = free.begin(); it != free.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n, o = it->first + n;
        free.erase(it);
        if (rest) free[o] = rest;
        used += n;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = (n + 255) & ~(size_t)255;
    used -= n;
    auto it = free.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free.erase(nx);
    }
    if (it != free.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free.erase(it);
      }
    }
  }
};

struct Request {
  uint64_t id;
  flb_request r;
  double t_submit;
};

struct Active {
  uint64_t id, tag, nsteps;
  flb_params p;
  double t_submit, t_admit;
  size_t off = 0, bytes = 0;
  SlotDesc desc;
  Stats stats;
  int cls = 1;  // compute class: 0 FP64, 1 FP32
};

static size_t request_bytes_of(const flb_params& p, int storage) {
  int wide = 0, tiles_x = 0, ntiles = 0;
  tile_shape(p.nx, p.ny, &wide, &tiles_x, &ntiles);
  size_t b = population_elems(p.nx, p.ny) * (storage == 0 ? 8 : 4);
  b = (b + 255) & ~(size_t)255;
  if (p.sample_every > 0) {
    b += ((size_t)ntiles * kNStat * 8 + 255) & ~(size_t)255;
    b += ((size_t)kServerBlocks * kNStat * 8 + 255) & ~(size_t)255;
  }
  b += 256;  // error flag and step
  return b;
}

}  // namespace flb

using namespace flb;

struct flb_server {
  flb_server_config cfg;
  hipStream_t st = nullptr;
  bool own_stream = false;
  char* arena = nullptr;
  FreeList fl;
  std::mutex mu;
  std::condition_variable cv, done_cv;
  std::deque<Request> queue;
  std::deque<flb_result> results;
  std::vector<Active> active;
  uint64_t next_id = 1, submitted = 0, completed = 0;
  uint64_t clock = 0;  // server steps so far (mirrors the device clock)
  // device tables per compute class
  SlotDesc* d_slots[2] = {nullptr, nullptr};
  int* d_prefix[2] = {nullptr, nullptr};
  uint64_t* d_clock = nullptr;
  double* d_open = nullptr;
  std::vector<SlotDesc> h_slots[2];
  std::vector<int> h_prefix[2];
  std::vector<int> members[2];  // indices into `active`
  int tiles[2] = {0, 0};
  std::chrono::steady_clock::time_point t_start;
  double busy = 0;
  std::thread worker;
  bool stop = false;
  int error = FLB_OK;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  }
  int admit_locked();
  int finish(const Active& a);
  int retire();
  int run_chunk();
  int pump(int max_chunks, int* did);
};

int flb_server::admit_locked() {
  while (!queue.empty() && (int)active.size() < cfg.max_slots) {
    Request& q = queue.front();
    const size_t bytes = request_bytes_of(q.r.p, cfg.precision);
    size_t off = 0;
    if (!fl.alloc(bytes, &off)) break;  // head waits for memory (FIFO)
    Active a;
    a.id = q.id;
    a.tag = q.r.tag;
    a.nsteps = q.r.nsteps;
    a.p = q.r.p;
    a.t_submit = q.t_submit;
    a.t_admit = now();
    a.off = off;
    a.bytes = bytes;
    std::memset(&a.desc, 0, sizeof(a.desc));
    fill_slot(&a.p, &a.desc);
    a.cls = compute_precision(&a.p);
    char* base = arena + off;
    size_t o = 0;
    auto take = [&](size_t n) {
      char* p = base + o;
      o += (n + 255) & ~(size_t)255;
      return p;
    };
    a.desc.pop = take(population_elems(a.p.nx, a.p.ny) * (cfg.precision == 0 ? 8 : 4));
    if (a.p.sample_every > 0) {
      a.desc.partials = (double*)take((size_t)a.desc.ntiles * kNStat * 8);
      a.stats.max_blocks = kServerBlocks;
    }
    double* records = a.p.sample_every > 0 ? (double*)take((size_t)kServerBlocks * kNStat * 8)
                                           : nullptr;
    a.desc.err = (int*)take(8);
    a.desc.err_step = (unsigned long long*)(a.desc.err + 2);
    a.desc.skz = nullptr;
    a.desc.t0 = (uint64_t)0 - clock;  // own time 0 at the current server clock
    a.desc.tend = a.nsteps;
    a.stats.reset(a.p.block_steps);
    // state: equilibrium (or thermal) start, cleared sums and flags
    const double mu = a.p.init == FLB_INIT_THERMAL ? 3.0 * a.p.kT : 0.0;
    hipError_t e = launch_init(cfg.precision == 0 ? 0 : 1, a.desc.pop, a.desc.pitch, nullptr,
                               nullptr, nullptr, a.p.rho0, a.p.ux0, a.p.uy0, slot_shift(a.desc), a.p.nx, a.p.ny,
                               mu, a.desc.k0, a.desc.k1, 0, 0, a.p.ny, st);
    if (e == hipSuccess && a.desc.partials) {
      e = launch_fill(a.desc.partials, (size_t)a.desc.ntiles * kNStat, 0.0, st);
      if (e == hipSuccess) e = launch_fill(records, (size_t)kServerBlocks * kNStat, 0.0, st);
    }
    if (e == hipSuccess) e = hipMemsetAsync(a.desc.err, 0, 4, st);
    if (e == hipSuccess) e = hipMemsetAsync(a.desc.err_step, 0xFF, 8, st);
    if (e != hipSuccess) {
      fl.release(off, bytes);  // the request stays queued
      return hip_fail(e, "request set-up");
    }
    active.push_back(a);
    queue.pop_front();
  }
  return FLB_OK;
}

static double* records_of(const Active& a, char* arena, int precision) {
  if (a.p.sample_every <= 0) return nullptr;
  size_t o = (population_elems(a.p.nx, a.p.ny) * (precision == 0 ? 8 : 4) + 255) & ~(size_t)255;
  o += ((size_t)a.desc.ntiles * kNStat * 8 + 255) & ~(size_t)255;
  return (double*)(arena + a.off + o);
}

// Reads the correlators of a request that reached its step count, queues its
// result and returns its memory.  On a HIP error nothing is released.
int flb_server::finish(const Active& a) {
  flb_result res;
  std::memset(&res, 0, sizeof(res));
  res.id = a.id;
  res.tag = a.tag;
  res.nsteps = a.nsteps;
  res.t_submit = a.t_submit;
  res.t_admit = a.t_admit;
  int err = 0;
  HIPC(hipMemcpy(&err, a.desc.err, 4, hipMemcpyDeviceToHost));
  res.status = err ? ((err & kErrInvalidVelocity) ? FLB_E_INVALID_VELOCITY : FLB_E_NONFINITE)
                   : FLB_OK;
  if (a.desc.partials && !err) {
    double* rec = records_of(a, arena, cfg.precision);
    HIPC(launch_open_sum(a.desc.partials, a.desc.ntiles, d_open, st));
    double open[kNStat];
    std::vector<double> recs((size_t)std::max<uint64_t>(a.stats.nb, 1) * kNStat);
    HIPC(hipMemcpyAsync(open, d_open, sizeof(open), hipMemcpyDeviceToHost, st));
    if (a.stats.nb)
      HIPC(hipMemcpyAsync(recs.data(), rec, a.stats.nb * kNStat * 8, hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    double mt0[81];
    fnorm_rows(a.p.ux0, a.p.uy0, mt0);
    finish_covariance(a.stats, recs, open, (uint64_t)a.p.nx * a.p.ny, mt0, &res.cov);
  }
  res.t_done = now();
  fl.release(a.off, a.bytes);
  {
    std::lock_guard<std::mutex> lk(mu);
    results.push_back(res);
    completed += 1;
  }
  done_cv.notify_all();
  return FLB_OK;
}

// Retires every request whose own time reached nsteps.  The list of active
// requests is replaced under the lock (other threads read its size); after a
// failure the requests not yet retired stay in it.
int flb_server::retire() {
  HIPC(hipStreamSynchronize(st));
  std::vector<Active> keep;
  int rc = FLB_OK;
  for (const Active& a : active) {
    if (rc == FLB_OK && a.desc.t0 + clock >= a.nsteps) {
      rc = finish(a);
      if (rc == FLB_OK) continue;
    }
    keep.push_back(a);
  }
  std::lock_guard<std::mutex> lk(mu);
  active.swap(keep);
  return rc;
}

// One chunk: upload the slot tables, launch chunk_steps batched steps, tick.
int flb_server::run_chunk() {
  const int K = cfg.chunk_steps;
  for (int c = 0; c < 2; ++c) {
    members[c].clear();
    h_slots[c].clear();
    h_prefix[c].assign(1, 0);
  }
  for (int i = 0; i < (int)active.size(); ++i) {
    const int c = active[i].cls;
    members[c].push_back(i);
    h_slots[c].push_back(active[i].desc);
    h_prefix[c].push_back(h_prefix[c].back() + active[i].desc.ntiles);
  }
  for (int c = 0; c < 2; ++c) {
    tiles[c] = h_prefix[c].back();
    if (members[c].empty()) continue;
    HIPC(hipMemcpyAsync(d_slots[c], h_slots[c].data(), h_slots[c].size() * sizeof(SlotDesc),
                        hipMemcpyHostToDevice, st));
    HIPC(hipMemcpyAsync(d_prefix[c], h_prefix[c].data(), h_prefix[c].size() * sizeof(int),
                        hipMemcpyHostToDevice, st));
  }
  const int storage = cfg.precision == 0 ? 0 : 1;
  for (int k = 0; k < K; ++k) {
    // the sampling variant only where some request of the class samples
    bool due[2] = {false, false};
    for (auto& a : active) {
      const uint64_t own = a.desc.t0 + clock + (uint64_t)k;
      due[a.cls] |= own < a.nsteps && a.p.sample_every > 0 && own % (uint64_t)a.p.sample_every == 0;
    }
    for (int c = 0; c < 2; ++c) {
      if (members[c].empty()) continue;
      const bool any_sample = due[c];
      // chunk_steps is even, so every request's own time has the parity of k
      HIPC(launch_step(storage, c, cfg.basis, any_sample, k & 1, d_slots[c], d_prefix[c],
                       (int)members[c].size(), tiles[c], d_clock, (uint32_t)k, LaunchCfg{},
                       st));
    }
    for (auto& a : active) {
      const uint64_t own = a.desc.t0 + clock + (uint64_t)k;
      if (own >= a.nsteps || a.p.sample_every <= 0) continue;
      if (own % (uint64_t)a.p.sample_every != 0) continue;
      HIPC(a.stats.after_sample((uint64_t)a.p.nx * a.p.ny, a.desc.partials, a.desc.ntiles,
                                records_of(a, arena, cfg.precision), st));
    }
  }
  HIPC(launch_tick(d_clock, (uint64_t)K, st));
  clock += (uint64_t)K;
  return FLB_OK;
}

int flb_server::pump(int max_chunks, int* did) {
  int n = 0;
  for (; n < max_chunks; ++n) {
    {
      std::lock_guard<std::mutex> lk(mu);
      const int rc = admit_locked();
      if (rc != FLB_OK) return rc;
    }
    if (active.empty()) break;
    const double t0 = now();
    int rc = run_chunk();
    if (rc != FLB_OK) return rc;
    rc = retire();
    if (rc != FLB_OK) return rc;
    std::lock_guard<std::mutex> lk(mu);
    busy += now() - t0;
  }
  if (did) *did = n;
  return FLB_OK;
}

extern "C" {

size_t flb_server_request_bytes(const flb_server_config* cfg, const flb_request* r) {
  if (!cfg || !r) return 0;
  flb_params p = r->p;
  p.precision = cfg->precision;
  p.basis = cfg->basis;
  if (flb::check_params(&p) != FLB_OK) return 0;
  return request_bytes_of(p, cfg->precision == FLB_FP64 ? 0 : 1);
}

int flb_server_create(const flb_server_config* cfg, void* hip_stream, flb_server** out) {
  if (!cfg || !out) return set_error(FLB_E_ARG, "null argument");
  *out = nullptr;
  if (cfg->max_slots <= 0 || cfg->chunk_steps <= 0 || cfg->mem_budget_bytes < 4096)
    return set_error(FLB_E_ARG, "bad server configuration");
  if (cfg->precision != FLB_FP64 && cfg->precision != FLB_FP32_SHIFTED)
    return set_error(FLB_E_ARG, "unknown precision");
  if (cfg->basis < 0 || cfg->basis > 2) return set_error(FLB_E_ARG, "unknown basis");
  flb_server* S = new (std::nothrow) flb_server();
  if (!S) return set_error(FLB_E_OOM, "host allocation");
  S->cfg = *cfg;
  S->cfg.chunk_steps += S->cfg.chunk_steps & 1;  // even: all requests share the streaming phase
  S->t_start = std::chrono::steady_clock::now();
  auto fail = [&](int rc) {
    flb_server_destroy(S);
    return rc;
  };
  hipError_t e;
  if (hip_stream) {
    S->st = (hipStream_t)hip_stream;
  } else {
    e = hipStreamCreateWithFlags(&S->st, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(hip_fail(e, "stream"));
    S->own_stream = true;
  }
  e = hipMalloc((void**)&S->arena, cfg->mem_budget_bytes);
  if (e != hipSuccess) return fail(set_error(FLB_E_OOM, "server arena of %zu bytes",
                                             cfg->mem_budget_bytes));
  S->fl.reset(cfg->mem_budget_bytes);
  for (int c = 0; c < 2; ++c) {
    e = hipMalloc((void**)&S->d_slots[c], (size_t)cfg->max_slots * sizeof(SlotDesc));
    if (e == hipSuccess) e = hipMalloc((void**)&S->d_prefix[c], (cfg->max_slots + 1) * sizeof(int));
    if (e != hipSuccess) return fail(set_error(FLB_E_OOM, "slot tables"));
  }
  e = hipMalloc((void**)&S->d_clock, 8);
  if (e == hipSuccess) e = hipMalloc((void**)&S->d_open, kNStat * sizeof(double));
  if (e != hipSuccess) return fail(set_error(FLB_E_OOM, "clock"));
  e = hipMemsetAsync(S->d_clock, 0, 8, S->st);
  if (e == hipSuccess) e = hipStreamSynchronize(S->st);
  if (e != hipSuccess) return fail(hip_fail(e, "clock init"));
  if (cfg->threaded) {
    S->worker = std::thread([S] {
      while (true) {
        {
          std::unique_lock<std::mutex> lk(S->mu);
          S->cv.wait(lk, [S] { return S->stop || !S->queue.empty() || !S->active.empty(); });
          if (S->stop) return;
        }
        int did = 0;
        const int rc = S->pump(1, &did);
        if (rc != FLB_OK) {
          std::lock_guard<std::mutex> lk(S->mu);
          S->error = rc;
          S->stop = true;
          S->done_cv.notify_all();
          return;
        }
        if (did == 0) {
          // nothing admissible: wait for a new submission
          std::unique_lock<std::mutex> lk(S->mu);
          S->cv.wait_for(lk, std::chrono::milliseconds(1));
        }
      }
    });
  }
  *out = S;
  return FLB_OK;
}

int flb_server_submit(flb_server* S, const flb_request* r, uint64_t* id) {
  if (!S || !r) return set_error(FLB_E_ARG, "null argument");
  flb_request q = *r;
  q.p.precision = S->cfg.precision;
  q.p.basis = S->cfg.basis;
  q.p.sk_every = 0;
  int rc = check_params(&q.p);
  if (rc != FLB_OK) return rc;
  if (q.nsteps == 0) return set_error(FLB_E_ARG, "request needs at least one step");
  if (q.nsteps >= (1ull << 62)) return set_error(FLB_E_ARG, "request of 2^62 steps or more");
  if (request_bytes_of(q.p, S->cfg.precision) > S->cfg.mem_budget_bytes)
    return set_error(FLB_E_ADMISSION, "request footprint exceeds the memory budget");
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return set_error(FLB_E_ADMISSION, "server stopped (error %d)", S->error);
    Request rq;
    rq.id = S->next_id++;
    rq.r = q;
    rq.t_submit = S->now();
    S->queue.push_back(rq);
    S->submitted += 1;
    if (id) *id = rq.id;
  }
  S->cv.notify_all();
  return FLB_OK;
}

int flb_server_pump(flb_server* S, int32_t max_chunks, int32_t* did_work) {
  if (!S) return set_error(FLB_E_ARG, "null server");
  if (S->cfg.threaded) return set_error(FLB_E_STATE, "threaded server pumps itself");
  int did = 0;
  const int rc = S->pump(max_chunks, &did);
  if (did_work) *did_work = did;
  return rc;
}

int flb_server_poll(flb_server* S, flb_result* out, int32_t max, int32_t* n) {
  if (!S || !n || (max > 0 && !out)) return set_error(FLB_E_ARG, "null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  int k = 0;
  while (k < max && !S->results.empty()) {
    out[k++] = S->results.front();
    S->results.pop_front();
  }
  *n = k;
  return S->error;
}

int flb_server_drain(flb_server* S) {
  if (!S) return set_error(FLB_E_ARG, "null server");
  if (!S->cfg.threaded) {
    while (true) {
      {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->completed == S->submitted) return FLB_OK;
      }
      int did = 0;
      const int rc = S->pump(1 << 20, &did);
      if (rc != FLB_OK) return rc;
      if (did == 0 && S->active.empty()) {
        std::lock_guard<std::mutex> lk(S->mu);
        if (!S->queue.empty()) return set_error(FLB_E_ADMISSION, "queued request cannot be admitted");
      }
    }
  }
  std::unique_lock<std::mutex> lk(S->mu);
  S->done_cv.wait(lk, [S] { return S->completed == S->submitted || S->stop; });
  return S->error;
}

int flb_server_stats(flb_server* S, int32_t* queued, int32_t* active, uint64_t* completed,
                     double* busy_seconds, double* wall_seconds) {
  if (!S) return set_error(FLB_E_ARG, "null server");
  std::lock_guard<std::mutex> lk(S->mu);
  if (queued) *queued = (int32_t)S->queue.size();
  if (active) *active = (int32_t)S->active.size();
  if (completed) *completed = S->completed;
  if (busy_seconds) *busy_seconds = S->busy;
  if (wall_seconds) *wall_seconds = S->now();
  return FLB_OK;
}

void flb_server_destroy(flb_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  if (S->worker.joinable()) S->worker.join();
  if (S->st) (void)hipStreamSynchronize(S->st);
  for (int c = 0; c < 2; ++c) {
    if (S->d_slots[c]) (void)hipFree(S->d_slots[c]);
    if (S->d_prefix[c]) (void)hipFree(S->d_prefix[c]);
  }
  if (S->d_clock) (void)hipFree(S->d_clock);
  if (S->d_open) (void)hipFree(S->d_open);
  if (S->arena) (void)hipFree(S->arena);
  if (S->own_stream && S->st) (void)hipStreamDestroy(S->st);
  delete S;
}

}  // extern "C"
