// Rollout / basis read-out: out[k] = U c_k for a block of coefficient
// columns, with U = S[:, :m] Q the logical basis (Q folded into the
// coefficients by the caller's coefficient kernel):
//     out[k*ldo + i] = sum_{j < m} S(i, j) * coefA[k*CMAX + j],
// S(i, j) stored at ((i/64)*ct + j)*64 + i%64 (64-row tiles).
// This is the O(N r) prediction of Sec. 2.3 (one read of the basis, one
// write per predicted state).  Each thread keeps one row of S in registers
// and streams the output rows; coefficient columns are wave-uniform and come
// through the scalar cache.
#include <hip/hip_runtime.h>

#include "odmd_internal.h"
#include "pass.h"
#include "storage.h"

namespace odmd {

template <typename TS, typename TO, int RB>
__global__ __launch_bounds__(256) void k_combine(CombineArgs c) {
  const DevState* __restrict__ st = c.st;
  const int ncols = st->m;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= c.n) return;
  const TS* __restrict__ Us = static_cast<const TS*>(c.Us);
  TO* __restrict__ out = static_cast<TO*>(c.out);
  double u[RB];
  const TS* __restrict__ T = Us + (i >> 6) * (int64_t)c.ct * 64 + (i & 63);
#pragma unroll
  for (int j = 0; j < RB; ++j) u[j] = j < ncols ? Storage<TS>::to_double(T[j * 64]) : 0.0;
  const int k0 = blockIdx.y * c.kb;
  const int k1 = min(c.K, k0 + c.kb);
  // coefficients are read-only for the launch: scalar loads via the
  // constant address space
  typedef const __attribute__((address_space(4))) double* cdp;
  cdp A = (cdp)st->coefA;
  for (int k = k0; k < k1; ++k) {
    asm volatile("" : "+s"(A));
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < RB; ++j) acc = __builtin_fma(u[j], A[k * CMAX + j], acc);
    out[(int64_t)k * c.ldo + i] = (TO)acc;
  }
}

template <typename TS, typename TO>
static hipError_t launch_t(const CombineArgs& c, int rb, hipStream_t s) {
  const dim3 grid((unsigned)((c.n + 255) / 256), (unsigned)((c.K + c.kb - 1) / c.kb)), block(256);
  switch (rb) {
    case 8: hipLaunchKernelGGL((k_combine<TS, TO, 8>), grid, block, 0, s, c); break;
    case 16: hipLaunchKernelGGL((k_combine<TS, TO, 16>), grid, block, 0, s, c); break;
    case 24: hipLaunchKernelGGL((k_combine<TS, TO, 24>), grid, block, 0, s, c); break;
    case 32: hipLaunchKernelGGL((k_combine<TS, TO, 32>), grid, block, 0, s, c); break;
    case 40: hipLaunchKernelGGL((k_combine<TS, TO, 40>), grid, block, 0, s, c); break;
    case 48: hipLaunchKernelGGL((k_combine<TS, TO, 48>), grid, block, 0, s, c); break;
    case 56: hipLaunchKernelGGL((k_combine<TS, TO, 56>), grid, block, 0, s, c); break;
    case 64: hipLaunchKernelGGL((k_combine<TS, TO, 64>), grid, block, 0, s, c); break;
    case 72: hipLaunchKernelGGL((k_combine<TS, TO, 72>), grid, block, 0, s, c); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_combine(const CombineArgs& c, int basis, int out_f32, int rb, hipStream_t s) {
  switch (basis) {
    case 0: return out_f32 ? launch_t<double, float>(c, rb, s) : launch_t<double, double>(c, rb, s);
    case 1: return out_f32 ? launch_t<float, float>(c, rb, s) : launch_t<float, double>(c, rb, s);
    case 2: return out_f32 ? launch_t<bf16, float>(c, rb, s) : launch_t<bf16, double>(c, rb, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace odmd
