// flb_runtime.hpp — internal declarations shared by the host-side sources of
// libflb (runtime, lattice/ensemble, server).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "flb.h"
#include "flb_kernels.hpp"

namespace flb {

// Above this background speed the FP32-storage path builds the local basis
// in FP64 (the Schur complement loses digits as u approaches the edge of the
// validity region).
constexpr double kFp32BasisMaxSpeed = 0.25;


int set_error(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
int check_params(const flb_params* p);
int compute_precision(const flb_params* p);
uint32_t row_pitch(int nx);
size_t population_elems(int nx, int ny);
void tile_shape(int nx, int ny, int* wide, int* tiles_x, int* ntiles);
void magic_div(uint32_t d, uint32_t* magic, uint32_t* shift);
void fill_slot(const flb_params* p, SlotDesc* d);
Shift9 slot_shift(const SlotDesc& d);
void hermite_rows(double m[81]);
double equilibrium(int i, double rho, double ux, double uy);
bool fnorm_rows(double ux, double uy, double mt[81]);

struct Stats {
  uint64_t tb_len = 0, tb_fill = 0, nb = 0, nsamples = 0;
  int max_blocks = kMaxTimeBlocks;  // record capacity (even)
  std::vector<uint64_t> rec_len;    // samples (time steps) per closed record
  void reset(int block_steps);
  hipError_t after_sample(uint64_t nsites, double* d_partials, int ntiles, double* d_records,
                          hipStream_t st);
  // Whether the next sample closes a time block without first merging
  // records; then close_counted does that sample's bookkeeping and returns
  // the record index, and the caller closes the block on the device.
  bool plain_close_next() const;
  uint64_t close_counted(uint64_t nsites);
  uint64_t block_samples(uint64_t b) const;
};

int finish_covariance(const Stats& S, const std::vector<double>& rec, const double* open,
                      uint64_t sites, const double mt0[81], flb_cov* out);

// launchers (flb_kernels.hip)
hipError_t launch_step(int storage, int compute, int basis, bool sample, int odd,
                       const SlotDesc* d_slots, const int* d_prefix, int nslots,
                       int total_tiles, const uint64_t* d_clock, uint32_t step_idx,
                       LaunchCfg cfg, hipStream_t st);
hipError_t launch_tick(uint64_t* d_clock, uint64_t n, hipStream_t st);
hipError_t launch_write_state(int storage, void* pop, uint32_t P, const double* f, int nx, int ny,
                              int odd, const Shift9& sh, int y0, int rows, hipStream_t st);
hipError_t launch_read_state(int storage, const void* pop, uint32_t P, double* f, int nx, int ny,
                             int odd, const Shift9& sh, int y0, int rows, hipStream_t st);
hipError_t launch_raw_state(int storage, void* pop, uint32_t P, void* buf, int nx, int ny, int odd,
                            int to_buf, int y0, int rows, hipStream_t st);
hipError_t launch_init(int storage, void* pop, uint32_t P, const double* rho, const double* ux,
                       const double* uy, double rho0, double ux0, double uy0, const Shift9& sh,
                       int nx, int ny, double mu, uint32_t k0, uint32_t k1, int odd, int y0,
                       int rows, hipStream_t st);
hipError_t launch_moments(int storage, const void* pop, uint32_t P, const double* B, double* out,
                          int nx, int ny, int odd, double rho0, double ux0, double uy0,
                          const Shift9& sh, int* err, int y0, int rows, hipStream_t st);
// The Fourier-coefficient readback: a grid of gx blocks of 256 columns by
// gy row groups, gx * gy <= max_blocks (returned), one partial per block
// at blockIdx.y * gx + blockIdx.x.
int fourier_mode_grid(int nx, int ny, int max_blocks, int* gx, int* gy);
hipError_t launch_fourier_mode(int storage, const void* pop, uint32_t P, double2* partial,
                               int max_blocks, int nx, int ny, int odd, int which, int kx, int ky,
                               double ux0, double uy0, hipStream_t st);
hipError_t launch_close_block(double* partials, int ntiles, double* record, hipStream_t st);
// n lattices of ntiles tiles each at once (device arrays of their partials
// and record bases; the record written at records[k] + record_offset)
hipError_t launch_close_block_many(double* const* partials, double* const* records,
                                  size_t record_offset, int n, int ntiles, hipStream_t st);
hipError_t launch_merge_blocks(double* rec, int nhalf, hipStream_t st);
hipError_t launch_open_sum(const double* partials, int ntiles, double* out, hipStream_t st);
hipError_t launch_fill(double* p, size_t n, double v, hipStream_t st);
hipError_t launch_stream_copy(const void* in, void* out, size_t n4, hipStream_t st);
hipError_t launch_stream_probe(int storage, void* pop, int nx, int ny, uint32_t pitch, int wide,
                               int tiles_x, int ntiles, int odd, hipStream_t st);
hipError_t sk_prepare(size_t max_lds);
hipError_t launch_sk_sample(int storage, void* z, void* zt, double* acc, int nx, int ny,
                            const void* twx, const void* twy, size_t max_lds, hipStream_t st);
// Whether rows of length n can be transformed (power of two that fits the
// LDS FFT, or short enough for the direct DFT).
int sk_transform_supported(int n, int storage, size_t max_lds);

// Bump allocator over one device allocation (256-byte aligned pieces).
struct Arena {
  char* base = nullptr;
  size_t used = 0, cap = 0;
  template <typename T>
  T* take(size_t count) {
    used = (used + 255) & ~(size_t)255;
    T* p = base ? reinterpret_cast<T*>(base + used) : nullptr;
    used += count * sizeof(T);
    return p;
  }
};

}  // namespace flb
