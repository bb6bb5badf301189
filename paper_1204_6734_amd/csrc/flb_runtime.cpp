// flb_runtime.cpp — host runtime behind the C ABI of include/flb.h:
// lattices (one slot) and ensembles (many slots of one shape), device
// memory arenas, time-block statistics, structure-factor pipeline,
// checkpoints and the measurement basis at (rho0, u0).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "flb.h"
#include "flb_kernels.hpp"
#include "flb_runtime.hpp"

namespace flb {

// ----------------------------------------------------------------- errors
static thread_local std::string g_err;

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return set_error(FLB_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIPC(expr)                                   \
  do {                                               \
    hipError_t e_ = (expr);                          \
    if (e_ != hipSuccess) return hip_fail(e_, #expr); \
  } while (0)

// ------------------------------------------------------------ host math
// Hermite rows of eq. (A3) and the D2Q9 weights of eq. (A2).
static const double kW[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
static const int kVXh[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int kVYh[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

void hermite_rows(double m[81]) {
  // rows as functions of the velocity: 1, sqrt3 vx, sqrt3 vy,
  // (3vx^2-3vy^2)/2, 3 vx vy, (3vx^2+3vy^2)/2 - 1, sqrt(3/2) vx (3vy^2-1),
  // sqrt(3/2) vy (3vx^2-1), (3vx^2-1)(3vy^2-1)/2
  for (int i = 0; i < 9; ++i) {
    const double x = kVXh[i], y = kVYh[i];
    const double hx = 3 * x * x - 1, hy = 3 * y * y - 1;
    m[0 * 9 + i] = 1;
    m[1 * 9 + i] = std::sqrt(3.0) * x;
    m[2 * 9 + i] = std::sqrt(3.0) * y;
    m[3 * 9 + i] = 1.5 * (x * x - y * y);
    m[4 * 9 + i] = 3 * x * y;
    m[5 * 9 + i] = 1.5 * (x * x + y * y) - 1;
    m[6 * 9 + i] = std::sqrt(1.5) * x * hy;
    m[7 * 9 + i] = std::sqrt(1.5) * y * hx;
    m[8 * 9 + i] = 0.5 * hx * hy;
  }
}

double equilibrium(int i, double rho, double ux, double uy) {
  const double c = ux * kVXh[i] + uy * kVYh[i];
  return rho * kW[i] * (1 + 3 * c + 4.5 * c * c - 1.5 * (ux * ux + uy * uy));
}

// f-norm rows at velocity u: m~ = L^-1 m with L L^T = m diag(g) m^T (the
// Gram-Schmidt of Sec. IV written as a Cholesky factorisation).  Returns
// false outside the validity region.
bool fnorm_rows(double ux, double uy, double mt[81]) {
  double m[81], g[9], G[81], L[81];
  hermite_rows(m);
  for (int i = 0; i < 9; ++i) {
    g[i] = equilibrium(i, 1.0, ux, uy);
    if (!(g[i] > 0)) return false;
  }
  for (int a = 0; a < 9; ++a)
    for (int b = 0; b < 9; ++b) {
      double s = 0;
      for (int i = 0; i < 9; ++i) s += m[a * 9 + i] * g[i] * m[b * 9 + i];
      G[a * 9 + b] = s;
    }
  std::memset(L, 0, sizeof(L));
  for (int j = 0; j < 9; ++j) {
    double d = G[j * 9 + j];
    for (int k = 0; k < j; ++k) d -= L[j * 9 + k] * L[j * 9 + k];
    if (!(d > 0)) return false;
    L[j * 9 + j] = std::sqrt(d);
    for (int i = j + 1; i < 9; ++i) {
      double s = G[i * 9 + j];
      for (int k = 0; k < j; ++k) s -= L[i * 9 + k] * L[j * 9 + k];
      L[i * 9 + j] = s / L[j * 9 + j];
    }
  }
  for (int c = 0; c < 9; ++c)
    for (int a = 0; a < 9; ++a) {
      double s = m[a * 9 + c];
      for (int k = 0; k < a; ++k) s -= L[a * 9 + k] * mt[k * 9 + c];
      mt[a * 9 + c] = s / L[a * 9 + a];
    }
  return true;
}

static bool valid_velocity(double ux, double uy) {
  for (int i = 0; i < 9; ++i)
    if (!(equilibrium(i, 1.0, ux, uy) > 0)) return false;
  return true;
}

int check_params(const flb_params* p) {
  if (!p) return set_error(FLB_E_ARG, "null parameters");
  if (p->nx < 3 || p->ny < 3) return set_error(FLB_E_ARG, "nx, ny must be >= 3");
  if ((uint64_t)p->nx + kTileX >= (1ull << 31) ||
      (uint64_t)row_pitch(p->nx) * (uint64_t)p->ny * 9ull >= (1ull << 32))
    return set_error(FLB_E_ARG, "lattice too large (9 ny nx, nx rounded up to 64, must fit "
                                "32 bits)");
  if (!(p->rho0 > 0) || !std::isfinite(p->rho0)) return set_error(FLB_E_ARG, "rho0 must be > 0");
  if (!(p->kT >= 0) || !std::isfinite(p->kT)) return set_error(FLB_E_ARG, "kT must be >= 0");
  for (int a = 0; a < 6; ++a)
    if (!(p->tau[a] > 0.5) || !std::isfinite(p->tau[a]))
      return set_error(FLB_E_ARG, "tau[%d] must be > 1/2", a);
  if (p->precision != FLB_FP64 && p->precision != FLB_FP32_SHIFTED)
    return set_error(FLB_E_ARG, "unknown precision");
  if (p->basis < 0 || p->basis > 2) return set_error(FLB_E_ARG, "unknown basis");
  if (p->init < 0 || p->init > 2) return set_error(FLB_E_ARG, "unknown init");
  if (p->sample_every < 0 || p->sk_every < 0 || p->block_steps < 0)
    return set_error(FLB_E_ARG, "negative sampling interval");
  if (!valid_velocity(p->ux0, p->uy0))
    return set_error(FLB_E_INVALID_VELOCITY, "u0 = (%g, %g) outside the validity region",
                     p->ux0, p->uy0);
  return FLB_OK;
}

// Compute precision of the collision: FP64 storage computes in FP64; FP32
// shifted storage computes in FP32 unless the background flow is fast, where
// the basis construction is carried out in FP64.
int compute_precision(const flb_params* p) {
  if (p->precision == FLB_FP64) return 0;
  const double u = std::sqrt(p->ux0 * p->ux0 + p->uy0 * p->uy0);
  return u > kFp32BasisMaxSpeed ? 0 : 1;
}

// Elements per plane row of the row-interleaved population storage: nx
// rounded up to whole wavefronts, so every plane row starts 256-byte
// aligned (FP32) and a wavefront's loads never straddle two plane rows.
uint32_t row_pitch(int nx) { return (uint32_t)((nx + kTileX - 1) / kTileX * kTileX); }

// Elements of a lattice's population storage (nine plane rows per row).
size_t population_elems(int nx, int ny) { return (size_t)9 * ny * row_pitch(nx); }

// Tile shape and count: 256 x 1 tiles (four wavefronts along a row) on rows
// of at least kWideTileMinNx sites, whose wavefronts then read longer
// stretches of one row (measured faster), else 64 x 4.
void tile_shape(int nx, int ny, int* wide, int* tiles_x, int* ntiles) {
  *wide = nx >= kWideTileMinNx ? 1 : 0;
  const int tw = *wide ? kTileX * kTileY : kTileX, th = *wide ? 1 : kTileY;
  *tiles_x = (nx + tw - 1) / tw;
  *ntiles = *tiles_x * ((ny + th - 1) / th);
}

// Division by d >= 1 as a multiply-shift (Granlund-Montgomery, round-up
// variant): m = ceil(2^k / d) with k = 32 + floor(log2 d) (31 + log2 d for a
// power of two, where the division is exact) fits 32 bits, and its error
// e = m d - 2^k < d keeps floor(t m / 2^k) = floor(t / d) for all t < 2^31.
void magic_div(uint32_t d, uint32_t* magic, uint32_t* shift) {
  const uint64_t dv = d;
  int lg = 0;
  while ((2ull << lg) <= dv) ++lg;  // floor(log2 d)
  const int k = (dv & (dv - 1)) == 0 ? 31 + lg : 32 + lg;
  *magic = (uint32_t)(((1ull << k) + dv - 1) / dv);
  *shift = (uint32_t)k;
}

void fill_slot(const flb_params* p, SlotDesc* d) {
  d->nx = p->nx;
  d->ny = p->ny;
  d->pitch = row_pitch(p->nx);
  tile_shape(p->nx, p->ny, &d->wide, &d->tiles_x, &d->ntiles);
  magic_div((uint32_t)d->tiles_x, &d->tx_magic, &d->tx_shift);
  magic_div(p->sample_every > 0 ? (uint32_t)p->sample_every : 1u, &d->se_magic, &d->se_shift);
  magic_div(p->sk_every > 0 ? (uint32_t)p->sk_every : 1u, &d->sk_magic, &d->sk_shift);
  d->k0 = (uint32_t)p->seed;
  d->k1 = (uint32_t)(p->seed >> 32);
  d->sample_every = p->sample_every;
  d->sk_every = p->sk_every;
  const double mu = 3.0 * p->kT;
  d->noise = mu > 0 ? 1 : 0;
  d->rho0 = p->rho0;
  d->ux0 = p->ux0;
  d->uy0 = p->uy0;
  d->rho0f = (float)p->rho0;
  d->ux0f = (float)p->ux0;
  d->uy0f = (float)p->uy0;
  d->one_tau = 1;
  for (int a = 0; a < 6; ++a) {
    const double tau = p->tau[a];
    d->rt[a] = 1.0 / tau;
    d->xc[a] = std::sqrt(mu * (2 * tau - 1)) / tau;
    d->rtf[a] = (float)d->rt[a];
    d->xcf[a] = (float)d->xc[a];
    if (tau != p->tau[0]) d->one_tau = 0;
  }
  d->xc2 = mu * (2 * p->tau[0] - 1) / (p->tau[0] * p->tau[0]);
  d->xc2f = (float)d->xc2;
  for (int i = 0; i < 9; ++i) {
    d->shift[i] = equilibrium(i, p->rho0, p->ux0, p->uy0);
    d->shiftf[i] = (float)d->shift[i];
  }
}

Shift9 slot_shift(const SlotDesc& d) {
  Shift9 s;
  for (int i = 0; i < 9; ++i) s.v[i] = d.shift[i];
  return s;
}

// ------------------------------------------------------------ statistics
void Stats::reset(int block_steps) {
  tb_len = block_steps > 0 ? (uint64_t)block_steps : 0;
  tb_fill = 0;
  nb = 0;
  nsamples = 0;
  rec_len.assign(max_blocks, 0);
}

// Bookkeeping after a correlator sample of `nsites` sites was enqueued: the
// open time block closes after tb_len samples (its partials are summed into
// record nb and cleared); a full record list merges neighbours pairwise and
// doubles the block length.
hipError_t Stats::after_sample(uint64_t nsites, double* d_partials, int ntiles, double* d_records,
                               hipStream_t st) {
  nsamples += nsites;
  if (tb_len == 0) return hipSuccess;
  if (++tb_fill < tb_len) return hipSuccess;
  if (rec_len.size() < (size_t)max_blocks) rec_len.assign(max_blocks, 0);
  if (nb == (uint64_t)max_blocks) {
    hipError_t e = launch_merge_blocks(d_records, max_blocks / 2, st);
    if (e != hipSuccess) return e;
    for (int b = 0; b < max_blocks / 2; ++b) rec_len[b] = rec_len[2 * b] + rec_len[2 * b + 1];
    nb = max_blocks / 2;
    tb_len *= 2;
  }
  hipError_t e = launch_close_block(d_partials, ntiles, d_records + nb * kNStat, st);
  rec_len[nb] = tb_fill;
  nb += 1;
  tb_fill = 0;
  return e;
}

bool Stats::plain_close_next() const {
  return tb_len != 0 && tb_fill + 1 == tb_len && nb < (uint64_t)max_blocks;
}

uint64_t Stats::close_counted(uint64_t nsites) {
  nsamples += nsites;
  if (rec_len.size() < (size_t)max_blocks) rec_len.assign(max_blocks, 0);
  const uint64_t b = nb;
  rec_len[b] = tb_fill + 1;
  nb += 1;
  tb_fill = 0;
  return b;
}

uint64_t Stats::block_samples(uint64_t b) const { return b < rec_len.size() ? rec_len[b] : 0; }

static void cov_from(const double* S, double n, double C[81]) {
  double m[9];
  for (int i = 0; i < 9; ++i) m[i] = S[i] / n;
  int k = 9;
  for (int i = 0; i < 9; ++i)
    for (int j = i; j < 9; ++j, ++k) {
      const double c = S[k] / n - m[i] * m[j];
      C[i * 9 + j] = c;
      C[j * 9 + i] = c;
    }
}

static void transform(const double B[81], const double C[81], double out[81]) {
  double T[81];
  for (int a = 0; a < 9; ++a)
    for (int j = 0; j < 9; ++j) {
      double s = 0;
      for (int i = 0; i < 9; ++i) s += B[a * 9 + i] * C[i * 9 + j];
      T[a * 9 + j] = s;
    }
  for (int a = 0; a < 9; ++a)
    for (int b = 0; b < 9; ++b) {
      double s = 0;
      for (int j = 0; j < 9; ++j) s += T[a * 9 + j] * B[b * 9 + j];
      out[a * 9 + b] = s;
    }
}

// Final correlators from the closed block records (nb x 54, host copy) and
// the open partial sums (54); standard errors from the spread of the
// per-record estimates.
int finish_covariance(const Stats& S, const std::vector<double>& rec, const double* open,
                      uint64_t sites, const double mt0[81], flb_cov* out) {
  std::memset(out, 0, sizeof(*out));
  out->nsamples = S.nsamples;
  out->nblocks = S.nb;
  if (S.nsamples == 0) return FLB_OK;
  double tot[kNStat];
  for (int v = 0; v < kNStat; ++v) tot[v] = 0;
  for (uint64_t b = 0; b < S.nb; ++b)
    for (int v = 0; v < kNStat; ++v) tot[v] += rec[b * kNStat + v];
  for (int v = 0; v < kNStat; ++v) tot[v] += open[v];
  const double n = (double)S.nsamples;
  for (int i = 0; i < 9; ++i) out->mean_df[i] = tot[i] / n;
  cov_from(tot, n, out->cov_f);
  double m[81];
  hermite_rows(m);
  transform(mt0, out->cov_f, out->cov_m_fnorm_u0);
  transform(m, out->cov_f, out->cov_m_hermite);
  if (S.nb >= 2) {
    double sf[81] = {0}, sf2[81] = {0}, sm[81] = {0}, sm2[81] = {0}, sh[81] = {0}, sh2[81] = {0};
    for (uint64_t b = 0; b < S.nb; ++b) {
      const double nbk = (double)S.block_samples(b) * (double)sites;
      double Cb[81], Mb[81], Hb[81];
      cov_from(&rec[b * kNStat], nbk, Cb);
      transform(mt0, Cb, Mb);
      transform(m, Cb, Hb);
      for (int k = 0; k < 81; ++k) {
        sf[k] += Cb[k];
        sf2[k] += Cb[k] * Cb[k];
        sm[k] += Mb[k];
        sm2[k] += Mb[k] * Mb[k];
        sh[k] += Hb[k];
        sh2[k] += Hb[k] * Hb[k];
      }
    }
    const double nb = (double)S.nb;
    auto se = [nb](double s1, double s2) {
      const double v = (s2 - s1 * s1 / nb) / (nb - 1);
      return std::sqrt(v > 0 ? v / nb : 0.0);
    };
    for (int k = 0; k < 81; ++k) {
      out->se_cov_f[k] = se(sf[k], sf2[k]);
      out->se_cov_m[k] = se(sm[k], sm2[k]);
      out->se_cov_m_hermite[k] = se(sh[k], sh2[k]);
    }
  } else {
    for (int k = 0; k < 81; ++k)
      out->se_cov_f[k] = out->se_cov_m[k] = out->se_cov_m_hermite[k] = NAN;
  }
  return FLB_OK;
}

}  // namespace flb

extern "C" const char* flb_last_error(void) { return flb::g_err.c_str(); }

namespace {
// Device time of `reps` runs of fn() after three unmeasured ones, on the
// null stream.
template <typename Fn>
hipError_t time_reps(int reps, Fn fn, float* ms) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  for (int w = 0; w < 3 && e == hipSuccess; ++w) e = fn();
  if (e == hipSuccess) e = hipEventRecord(e0, 0);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = fn();
  if (e == hipSuccess) e = hipEventRecord(e1, 0);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return e;
}
}  // namespace

extern "C" int flb_copy_probe(int32_t nx, int32_t ny, int32_t precision, int32_t reps,
                              double* ms_per_pass) {
  using flb::set_error;
  flb_params p;
  std::memset(&p, 0, sizeof(p));
  p.nx = nx;
  p.ny = ny;
  p.rho0 = 1.0;
  for (int a = 0; a < 6; ++a) p.tau[a] = 1.0;
  p.precision = precision;
  if (reps < 1 || reps > 1000 || !ms_per_pass)
    return set_error(FLB_E_ARG, "copy probe: bad arguments");
  const int rc = flb::check_params(&p);
  if (rc != FLB_OK) return rc;
  const int storage = precision == FLB_FP64 ? 0 : 1;
  const size_t bytes = flb::population_elems(nx, ny) * (storage == 0 ? 8 : 4);
  int wide = 0, tiles_x = 0, ntiles = 0;
  flb::tile_shape(nx, ny, &wide, &tiles_x, &ntiles);
  const uint32_t pitch = flb::row_pitch(nx);
  void* a = nullptr;
  if (hipMalloc(&a, bytes) != hipSuccess) return set_error(FLB_E_OOM, "copy probe");
  struct Free {
    void* a;
    ~Free() { (void)hipFree(a); }
  } fr{a};
  hipError_t e = hipMemset(a, 0, bytes);
  float ms = 0.f;
  // one even and one odd pass per repetition
  if (e == hipSuccess)
    e = time_reps(reps, [&]() {
      hipError_t r = flb::launch_stream_probe(storage, a, nx, ny, pitch, wide, tiles_x, ntiles, 0,
                                              0);
      if (r == hipSuccess)
        r = flb::launch_stream_probe(storage, a, nx, ny, pitch, wide, tiles_x, ntiles, 1, 0);
      return r;
    }, &ms);
  if (e != hipSuccess) return flb::hip_fail(e, "copy probe");
  *ms_per_pass = ms / (2.0 * reps);
  return FLB_OK;
}

extern "C" int flb_stream_copy_probe(uint64_t bytes, int32_t reps, double* ms_per_copy) {
  using flb::set_error;
  if (bytes == 0 || bytes % 16 != 0 || bytes >= (1ull << 40) || reps < 1 || reps > 1000 ||
      !ms_per_copy)
    return set_error(FLB_E_ARG, "stream copy probe: bad arguments");
  void *a = nullptr, *b = nullptr;
  if (hipMalloc(&a, bytes) != hipSuccess) return set_error(FLB_E_OOM, "stream copy probe");
  if (hipMalloc(&b, bytes) != hipSuccess) {
    (void)hipFree(a);
    return set_error(FLB_E_OOM, "stream copy probe");
  }
  struct Free {
    void *a, *b;
    ~Free() {
      (void)hipFree(a);
      (void)hipFree(b);
    }
  } fr{a, b};
  hipError_t e = hipMemset(a, 0, bytes);
  float ms = 0.f;
  if (e == hipSuccess)
    e = time_reps(reps, [&]() { return flb::launch_stream_copy(a, b, bytes / 16, 0); }, &ms);
  if (e != hipSuccess) return flb::hip_fail(e, "stream copy probe");
  *ms_per_copy = ms / reps;
  return FLB_OK;
}
