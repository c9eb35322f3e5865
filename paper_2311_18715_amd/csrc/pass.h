// Host-side declarations of the kernel launchers (one per .hip file).
#pragma once
#include <hip/hip_runtime.h>

#include "odmd_internal.h"

namespace odmd {

struct PassArgs {
  void* Us;             // stored basis, column-major, leading dim ld
  void* Es;             // stored residual
  const void* x;        // snapshot x_k (io type)
  const void* y;        // snapshot x_k+1 (io type)
  double* partials;     // nblk x PW
  const DevState* st;
  int64_t n, ld;
  int nblk, tiles;      // workgroups, 256-row tiles
};

// rb: rank bucket (multiple of 8, >= r_max of the stream)
hipError_t launch_pass(const PassArgs& p, int basis_f64, int rb, hipStream_t s);

struct CoreArgs {
  DevState* st;
  const double* partials;
  int nblk;
  int r_max;
  int basis_f32;        // also keep an FP32 copy of the rotation
  int jacobi_only;      // skip the secular solver (diagnostics)
};
hipError_t launch_core(const CoreArgs& c, hipStream_t s);

struct CombineArgs {
  const DevState* st;   // coefficients coefA / coefB and the basis layout
  const void* Us;       // stored basis
  const void* Es;       // stored residual
  void* out;            // out[k*ldo + i], k < K
  int64_t n, ld, ldo;
  int K, kb;            // columns, columns per workgroup row of the grid
};
// out type: 0 = FP64, 1 = FP32; basis_f64 selects the stored type
hipError_t launch_combine(const CombineArgs& c, int basis_f64, int out_f32, int rb, hipStream_t s);

hipError_t launch_basis_coef(DevState* st, hipStream_t s);
hipError_t launch_eig(DevState* st, hipStream_t s);
hipError_t launch_predict_coef(DevState* st, int k0, int steps, hipStream_t s);

}  // namespace odmd
