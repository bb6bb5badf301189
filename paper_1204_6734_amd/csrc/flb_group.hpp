// flb_group.hpp — a group of lattices ("slots") advanced by one batched step
// launch per step on one stream (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <utility>
#include <vector>

#include "flb.h"
#include "flb_kernels.hpp"
#include "flb_runtime.hpp"

namespace flb {

constexpr int kModeBlocks = 1024;

struct Group {
  std::vector<flb_params> P;
  std::vector<SlotDesc> hdesc;
  std::vector<int> prefix;
  int storage = 1, compute = 1, basis = 0, total_tiles = 0;
  // Members whose background speed needs the FP64 collision (FP32 storage,
  // |u0| > 0.25) form their own launch class, so that every member computes
  // exactly as it would alone.  Class c: compute precision ccompute[c], the
  // device descriptors d_slots + cfirst[c] (members in class order), tile
  // prefix sums d_prefix + cfirst[c] + c, ccount[c] members and ctiles[c]
  // tiles.
  int nclass = 1;
  int ccompute[2] = {1, 0}, cfirst[2] = {0, 0}, ccount[2] = {0, 0}, ctiles[2] = {0, 0};
  std::vector<int> corder;  // device position -> member
  hipStream_t st = nullptr;
  bool own_stream = false, own_mem = false;
  void* dev = nullptr;
  size_t need_bytes = 0;
  size_t max_lds = 65536;
  // device arrays
  SlotDesc* d_slots = nullptr;
  int* d_prefix = nullptr;
  uint64_t* d_clock = nullptr;
  int* d_err = nullptr;
  unsigned long long* d_err_step = nullptr;
  double* d_open = nullptr;
  double* d_B = nullptr;
  double2* d_mode = nullptr;
  double* d_io = nullptr;
  int band_rows = 1;
  std::vector<void*> pop;
  std::vector<double*> d_partials, d_records;
  double** d_close = nullptr;  // [2n] device copies: every slot's partials, then its records
  // structure factor: complex planes and twiddles in the storage precision
  void* d_z = nullptr;
  void* d_zt = nullptr;
  double* d_skacc = nullptr;  // [5][nx/2 + 1][ny]
  void* d_twx = nullptr;
  void* d_twy = nullptr;
  // host state
  uint64_t t = 0, nsk = 0;
  int64_t err_step_host = -1;
  std::vector<Stats> stats;
  std::vector<std::vector<double>> mt0;
  // launch shape of the step kernel
  LaunchCfg launch;
  int device = 0;
  // graphs
  int graph_chunk = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  // profiling
  bool profiling = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  double prof_ms = 0;
  uint64_t prof_launches = 0;

  Group() = default;
  Group(const Group&) = delete;
  Group& operator=(const Group&) = delete;
  ~Group();

  void layout(Arena& a);
  int init(const flb_params* ps, int n, void* stream, void* dev_buf, size_t dev_bytes);
  bool sample_due(int s, uint64_t tt) const;
  bool sk_due(int s, uint64_t tt) const;
  int after_step(uint64_t tt, bool replayed = false);
  bool lockstep_close(uint64_t tt) const;
  int launch_one(uint32_t k, bool sample, int odd);
  hipError_t launch_classes(uint32_t k, bool sample, int odd, LaunchCfg c);
  bool graph_friendly() const;
  uint64_t steps_to_close() const;
  int capture_graph();
  int step(uint64_t nsteps);
  int sync();
  int read_populations(int s, double* f);
  int read_rows(int s, int y0, int nrows, double* f);
  int set_populations(int s, const double* f, uint64_t tnew);
  int set_fields(int s, const double* rho, const double* ux, const double* uy);
  int read_moments(int s, int at, double* m);
  int read_covariance(int s, flb_cov* out);
  int reset_stats();
  int read_structure_factor(int which, double* out);
  int read_fourier_mode(int which, int kx, int ky, double out[2]);
  size_t checkpoint_bytes() const;
  int checkpoint(void* host, size_t bytes);
  int restore(const void* host, size_t bytes);
  int kernel_time(double* ms, uint64_t* launches);
  void drop_graph();
  // accumulator entries of one structure factor: the half plane kx <= nx/2
  size_t sk_half() const { return (size_t)(P[0].nx / 2 + 1) * P[0].ny; }
  int set_launch(const flb_launch_config* c);
  int autotune(int reps, flb_launch_config* results, int max_results, int* n_results);
};

// Launch shape an earlier autotune in this process chose for groups like g
// (same device, storage, compute, basis and tile count), else the default.
LaunchCfg tuned_launch(const Group& g);

}  // namespace flb
