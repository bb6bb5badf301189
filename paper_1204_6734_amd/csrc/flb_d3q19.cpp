// flb_d3q19.cpp — D3Q19 lattices: host runtime and C ABI (flb3_*).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <utility>
#include <vector>

#include "d3q19_tables.hpp"
#include "flb.h"
#include "flb_d3q19.hpp"
#include "flb_runtime.hpp"

namespace flb {
namespace d3q19 {

#define HIPC(expr)                                    \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return hip_fail(e_, #expr); \
  } while (0)

static double equilibrium3(int i, double rho, const double u[3]) {
  const double cu = kC3[i][0] * u[0] + kC3[i][1] * u[1] + kC3[i][2] * u[2];
  const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  return kW3[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
}

static int check3(const flb3_params* p) {
  if (!p) return set_error(FLB_E_ARG, "null parameters");
  if (p->nx < 3 || p->ny < 3 || p->nz < 3) return set_error(FLB_E_ARG, "nx, ny, nz must be >= 3");
  if ((uint64_t)p->nx * p->ny * p->nz * 19ull >= (1ull << 32))
    return set_error(FLB_E_ARG, "lattice too large (19 nx ny nz must fit 32 bits)");
  if (!(p->rho0 > 0) || !std::isfinite(p->rho0)) return set_error(FLB_E_ARG, "rho0 must be > 0");
  if (!(p->kT >= 0) || !std::isfinite(p->kT)) return set_error(FLB_E_ARG, "kT must be >= 0");
  for (int a = 0; a < 15; ++a)
    if (!(p->tau[a] > 0.5) || !std::isfinite(p->tau[a]))
      return set_error(FLB_E_ARG, "tau[%d] must be > 1/2", a);
  if (p->precision != FLB_FP64 && p->precision != FLB_FP32_SHIFTED)
    return set_error(FLB_E_ARG, "unknown precision");
  if (p->basis != FLB_BASIS_FNORM_LOCAL && p->basis != FLB_BASIS_HERMITE)
    return set_error(FLB_E_ARG, "D3Q19 supports the local f-norm and the Hermite rows");
  if (p->sample_every < 0 || p->block_steps < 0)
    return set_error(FLB_E_ARG, "negative sampling interval");
  const double u[3] = {p->ux0, p->uy0, p->uz0};
  for (int i = 0; i < 19; ++i)
    if (!(equilibrium3(i, 1.0, u) > 0))
      return set_error(FLB_E_INVALID_VELOCITY, "u0 outside the validity region");
  return FLB_OK;
}

struct Lattice3 {
  flb3_params p{};
  int storage = 1;
  size_t N = 0;
  Desc3 h{};
  Desc3* d_desc = nullptr;
  char* dev = nullptr;
  uint64_t* d_clock = nullptr;
  int* d_err = nullptr;
  unsigned long long* d_err_step = nullptr;
  double* d_records = nullptr;
  double* d_open = nullptr;
  hipStream_t st = nullptr;
  bool own_stream = false;
  uint64_t t = 0;
  int64_t err_step_host = -1;
  // time blocks of the correlator sums
  static constexpr int kMaxBlocks = 1024;
  uint64_t tb_len = 0, tb_fill = 0, nb = 0, nsamples = 0;
  std::vector<uint64_t> rec_len;
  // profiling
  bool profiling = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  double prof_ms = 0;
  uint64_t prof_launches = 0;

  ~Lattice3() {
    if (st) (void)hipStreamSynchronize(st);
    for (auto& e : events) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    if (dev) (void)hipFree(dev);
    if (own_stream && st) (void)hipStreamDestroy(st);
  }

  int init(const flb3_params* pp, void* stream) {
    int rc = check3(pp);
    if (rc != FLB_OK) return rc;
    p = *pp;
    storage = p.precision == FLB_FP64 ? 0 : 1;
    N = (size_t)p.nx * p.ny * p.nz;
    const size_t es = storage == 0 ? sizeof(double) : sizeof(float);
    h.nx = p.nx;
    h.ny = p.ny;
    h.nz = p.nz;
    h.tiles_x = (p.nx + 63) / 64;
    h.tiles_xy = h.tiles_x * ((p.ny + 3) / 4);
    h.ntiles = h.tiles_xy * p.nz;
    h.k0 = (uint32_t)p.seed;
    h.k1 = (uint32_t)(p.seed >> 32);
    h.sample_every = p.sample_every;
    const double mu = 3.0 * p.kT;
    h.noise = mu > 0 ? 1 : 0;
    h.rho0 = p.rho0;
    h.u0[0] = p.ux0;
    h.u0[1] = p.uy0;
    h.u0[2] = p.uz0;
    h.rho0f = (float)p.rho0;
    for (int a = 0; a < 3; ++a) h.u0f[a] = (float)h.u0[a];
    h.one_tau = 1;
    for (int a = 0; a < 15; ++a) {
      h.rt[a] = 1.0 / p.tau[a];
      h.xc[a] = std::sqrt(mu * (2 * p.tau[a] - 1)) / p.tau[a];
      h.rtf[a] = (float)h.rt[a];
      h.xcf[a] = (float)h.xc[a];
      if (p.tau[a] != p.tau[0]) h.one_tau = 0;
    }
    h.xc2 = mu * (2 * p.tau[0] - 1) / (p.tau[0] * p.tau[0]);
    h.xc2f = (float)h.xc2;
    for (int i = 0; i < 19; ++i) h.shift[i] = equilibrium3(i, p.rho0, h.u0);
    // one allocation: descriptor, clock, error flags, populations, partials,
    // time-block records, open sums
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t part = p.sample_every > 0 ? (size_t)h.ntiles * kNStat3 : 0;
    const size_t rec = p.sample_every > 0 ? (size_t)kMaxBlocks * kNStat3 : 0;
    const size_t sizes[] = {sizeof(Desc3), sizeof(uint64_t), sizeof(int),
                            sizeof(unsigned long long), 19 * N * es, part * sizeof(double),
                            rec * sizeof(double), kNStat3 * sizeof(double)};
    size_t total = 0;
    for (size_t b : sizes) total += up(b);
    hipError_t e = hipMalloc((void**)&dev, total);
    if (e != hipSuccess) {
      dev = nullptr;
      return set_error(FLB_E_OOM, "hipMalloc(%zu): %s", total, hipGetErrorString(e));
    }
    char* q = dev;
    d_desc = (Desc3*)q;
    q += up(sizes[0]);
    d_clock = (uint64_t*)q;
    q += up(sizes[1]);
    d_err = (int*)q;
    q += up(sizes[2]);
    d_err_step = (unsigned long long*)q;
    q += up(sizes[3]);
    h.pop = q;
    q += up(sizes[4]);
    h.partials = part ? (double*)q : nullptr;
    q += up(sizes[5]);
    d_records = rec ? (double*)q : nullptr;
    q += up(sizes[6]);
    d_open = (double*)q;
    h.err = d_err;
    h.err_step = d_err_step;
    if (stream) {
      st = (hipStream_t)stream;
    } else {
      HIPC(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      own_stream = true;
    }
    HIPC(hipMemcpyAsync(d_desc, &h, sizeof(Desc3), hipMemcpyHostToDevice, st));
    HIPC(hipMemsetAsync(d_clock, 0, sizeof(uint64_t), st));
    HIPC(hipMemsetAsync(d_err, 0, sizeof(int), st));
    HIPC(hipMemsetAsync(d_err_step, 0xFF, sizeof(unsigned long long), st));
    // equilibrium start: the shifted populations are zero
    HIPC(hipMemsetAsync(h.pop, 0, 19 * N * es, st));
    if (part) HIPC(launch_fill3(h.partials, part, st));
    reset_blocks();
    HIPC(hipStreamSynchronize(st));
    return FLB_OK;
  }

  void reset_blocks() {
    tb_len = p.block_steps > 0 ? (uint64_t)p.block_steps : 0;
    tb_fill = 0;
    nb = 0;
    nsamples = 0;
    rec_len.assign(kMaxBlocks, 0);
  }

  int after_sample() {
    nsamples += N;
    if (tb_len == 0 || ++tb_fill < tb_len) return FLB_OK;
    if (nb == (uint64_t)kMaxBlocks) {
      HIPC(launch_merge_blocks3(d_records, kMaxBlocks / 2, st));
      for (int b = 0; b < kMaxBlocks / 2; ++b) rec_len[b] = rec_len[2 * b] + rec_len[2 * b + 1];
      nb = kMaxBlocks / 2;
      tb_len *= 2;
    }
    HIPC(launch_close_block3(h.partials, h.ntiles, d_records + nb * kNStat3, st));
    rec_len[nb] = tb_fill;
    nb += 1;
    tb_fill = 0;
    return FLB_OK;
  }

  int step(uint64_t n) {
    const uint64_t chunk_max = 1ull << 30;
    uint64_t done = 0;
    while (done < n) {
      const uint64_t chunk = std::min(n - done, chunk_max);
      for (uint64_t k = 0; k < chunk; ++k) {
        const uint64_t tt = t + k;
        const bool sample = p.sample_every > 0 && tt % (uint64_t)p.sample_every == 0;
        std::pair<hipEvent_t, hipEvent_t> ev{};
        if (profiling) {
          HIPC(hipEventCreate(&ev.first));
          HIPC(hipEventCreate(&ev.second));
          HIPC(hipEventRecord(ev.first, st));
        }
        HIPC(launch_step3(storage, p.basis == FLB_BASIS_HERMITE ? 1 : 0, h.one_tau != 0, sample,
                          (int)(tt & 1), h.ntiles, d_desc, d_clock, (uint32_t)k, st));
        if (profiling) {
          HIPC(hipEventRecord(ev.second, st));
          events.push_back(ev);
          prof_launches += 1;
        }
        if (sample) {
          const int rc = after_sample();
          if (rc != FLB_OK) return rc;
        }
      }
      HIPC(launch_tick(d_clock, chunk, st));
      t += chunk;
      done += chunk;
    }
    return FLB_OK;
  }

  int sync() {
    HIPC(hipStreamSynchronize(st));
    int err = 0;
    unsigned long long es = 0;
    HIPC(hipMemcpy(&err, d_err, sizeof(int), hipMemcpyDeviceToHost));
    HIPC(hipMemcpy(&es, d_err_step, sizeof(es), hipMemcpyDeviceToHost));
    if (err) {
      err_step_host = (int64_t)es;
      if (err & kErrInvalidVelocity)
        return set_error(FLB_E_INVALID_VELOCITY, "a site left the validity region at step %llu",
                         es);
      return set_error(FLB_E_NONFINITE, "non-finite populations at step %llu", es);
    }
    return FLB_OK;
  }

  int io(double* f, int to_storage) {
    double* d_f = nullptr;
    hipError_t e = hipMalloc((void**)&d_f, 19 * N * sizeof(double));
    if (e != hipSuccess) return set_error(FLB_E_OOM, "populations staging");
    struct Free {
      double* p;
      ~Free() { (void)hipFree(p); }
    } fr{d_f};
    if (to_storage) HIPC(hipMemcpy(d_f, f, 19 * N * sizeof(double), hipMemcpyHostToDevice));
    HIPC(launch_io3(storage, h.pop, d_f, h, (int)(t & 1), to_storage, st));
    HIPC(hipStreamSynchronize(st));
    if (!to_storage) HIPC(hipMemcpy(f, d_f, 19 * N * sizeof(double), hipMemcpyDeviceToHost));
    return FLB_OK;
  }

  int read_covariance(flb3_cov* out) {
    int rc = sync();
    if (rc != FLB_OK) return rc;
    std::memset(out, 0, sizeof(*out));
    out->nsamples = nsamples;
    out->nblocks = nb;
    if (!h.partials || nsamples == 0) return FLB_OK;
    std::vector<double> rec(nb * kNStat3), open(kNStat3);
    if (nb) HIPC(hipMemcpy(rec.data(), d_records, rec.size() * sizeof(double),
                           hipMemcpyDeviceToHost));
    HIPC(launch_open_sum3(h.partials, h.ntiles, d_open, st));
    HIPC(hipStreamSynchronize(st));
    HIPC(hipMemcpy(open.data(), d_open, kNStat3 * sizeof(double), hipMemcpyDeviceToHost));
    std::vector<double> tot(open);
    for (uint64_t b = 0; b < nb; ++b)
      for (int v = 0; v < kNStat3; ++v) tot[v] += rec[b * kNStat3 + v];
    cov_from(tot.data(), (double)nsamples, out->mean_df, out->cov_f);
    if (nb >= 2) {
      double s1[361] = {0}, s2[361] = {0};
      for (uint64_t b = 0; b < nb; ++b) {
        double mean[19], c[361];
        cov_from(&rec[b * kNStat3], (double)rec_len[b] * (double)N, mean, c);
        for (int k = 0; k < 361; ++k) {
          s1[k] += c[k];
          s2[k] += c[k] * c[k];
        }
      }
      const double n = (double)nb;
      for (int k = 0; k < 361; ++k) {
        const double v = (s2[k] - s1[k] * s1[k] / n) / (n - 1);
        out->se_cov_f[k] = std::sqrt(v > 0 ? v / n : 0.0);
      }
    } else {
      for (int k = 0; k < 361; ++k) out->se_cov_f[k] = NAN;
    }
    return FLB_OK;
  }

  static void cov_from(const double* S, double n, double mean[19], double C[361]) {
    for (int i = 0; i < 19; ++i) mean[i] = S[i] / n;
    int q = 19;
    for (int i = 0; i < 19; ++i)
      for (int j = i; j < 19; ++j, ++q) {
        const double c = S[q] / n - mean[i] * mean[j];
        C[i * 19 + j] = c;
        C[j * 19 + i] = c;
      }
  }

  int reset_stats() {
    HIPC(hipStreamSynchronize(st));
    if (h.partials) HIPC(launch_fill3(h.partials, (size_t)h.ntiles * kNStat3, st));
    reset_blocks();
    return FLB_OK;
  }

  int kernel_time(double* ms, uint64_t* launches) {
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
    if (ms) *ms = prof_ms + tot;
    if (launches) *launches = prof_launches;
    prof_ms = 0;
    prof_launches = 0;
    return FLB_OK;
  }
};

}  // namespace d3q19
}  // namespace flb

struct flb3_lattice {
  flb::d3q19::Lattice3 L;
};

extern "C" {

#define NEED3(h) \
  if (!(h)) return flb::set_error(FLB_E_ARG, "null handle")

int flb3_lattice_create(const flb3_params* p, void* hip_stream, flb3_lattice** out) {
  if (!out) return flb::set_error(FLB_E_ARG, "null output handle");
  *out = nullptr;
  flb3_lattice* L = new (std::nothrow) flb3_lattice();
  if (!L) return flb::set_error(FLB_E_OOM, "host allocation");
  const int rc = L->L.init(p, hip_stream);
  if (rc != FLB_OK) {
    delete L;
    return rc;
  }
  *out = L;
  return FLB_OK;
}
int flb3_lattice_set_populations(flb3_lattice* L, const double* f, uint64_t t) {
  NEED3(L);
  if (!f) return flb::set_error(FLB_E_ARG, "null populations");
  hipError_t e = hipStreamSynchronize(L->L.st);
  if (e != hipSuccess) return flb::hip_fail(e, "sync");
  L->L.t = t;
  e = hipMemcpy(L->L.d_clock, &t, sizeof(uint64_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) return flb::hip_fail(e, "clock");
  return L->L.io(const_cast<double*>(f), 1);
}
int flb3_lattice_step(flb3_lattice* L, uint64_t n) {
  NEED3(L);
  return L->L.step(n);
}
int flb3_lattice_sync(flb3_lattice* L) {
  NEED3(L);
  return L->L.sync();
}
int flb3_lattice_read_populations(flb3_lattice* L, double* f) {
  NEED3(L);
  if (!f) return flb::set_error(FLB_E_ARG, "null output");
  const int rc = L->L.sync();
  if (rc != FLB_OK) return rc;
  return L->L.io(f, 0);
}
int flb3_lattice_read_covariance(flb3_lattice* L, flb3_cov* out) {
  NEED3(L);
  if (!out) return flb::set_error(FLB_E_ARG, "null output");
  return L->L.read_covariance(out);
}
int flb3_lattice_reset_stats(flb3_lattice* L) {
  NEED3(L);
  return L->L.reset_stats();
}
uint64_t flb3_lattice_time(flb3_lattice* L) { return L ? L->L.t : 0; }
int64_t flb3_lattice_error_step(flb3_lattice* L) { return L ? L->L.err_step_host : -1; }
int flb3_lattice_profile(flb3_lattice* L, int32_t on) {
  NEED3(L);
  L->L.profiling = on != 0;
  return FLB_OK;
}
int flb3_lattice_kernel_time(flb3_lattice* L, double* ms, uint64_t* launches) {
  NEED3(L);
  return L->L.kernel_time(ms, launches);
}
void flb3_lattice_destroy(flb3_lattice* L) { delete L; }

}  // extern "C"
