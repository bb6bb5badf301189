// flb_d3q19.hpp — device descriptor and launchers of the D3Q19 lattice
// (internal; the C ABI is in include/flb.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace flb {
namespace d3q19 {

constexpr int kNStat3 = 19 + 190;  // first moments + products i <= j

struct Desc3 {
  void* pop;                     // [19][nz][ny][nx] shifted populations
  double* partials;              // [ntiles][kNStat3] open time-block sums, or null
  int* err;
  unsigned long long* err_step;
  int nx, ny, nz, tiles_x, tiles_xy, ntiles;
  uint32_t k0, k1;
  int sample_every, noise;
  int one_tau, pad_;             // all fifteen relaxation times equal
  double rho0, u0[3];
  double rt[15], xc[15];         // 1/tau, sqrt(mu (2 tau - 1)) / tau
  double xc2;                    // mu (2 tau - 1) / tau^2 = xc^2 when one_tau
  double shift[19];              // f_i^0(rho0, u0)
  float rho0f, u0f[3], rtf[15], xcf[15], xc2f;  // the same in FP32
};

hipError_t launch_step3(int storage, int basis, bool one_tau, bool sample, int odd, int ntiles,
                        const Desc3* d, const uint64_t* clock, uint32_t k, hipStream_t st);
hipError_t launch_io3(int storage, void* pop, double* f, const Desc3& d, int odd, int to_storage,
                      hipStream_t st);
hipError_t launch_close_block3(double* partials, int ntiles, double* record, hipStream_t st);
hipError_t launch_merge_blocks3(double* rec, int nhalf, hipStream_t st);
hipError_t launch_open_sum3(const double* partials, int ntiles, double* out, hipStream_t st);
hipError_t launch_fill3(double* p, size_t n, hipStream_t st);

}  // namespace d3q19
}  // namespace flb
