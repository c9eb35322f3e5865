// Rollout / basis read-out: out[k] = U c_k for a block of coefficient
// columns, with U the logical basis (Us G + Es g^T when a rotation is
// pending, folded into the coefficients by the caller's coefficient kernel):
//     out[k*ldo + i] = sum_j Us(i, j) * coefA[k*RMAX + j] + Es[i] * coefB[k],
// Us(i, j) stored at ((i/64)*ct + j)*64 + i%64 (64-row tiles).
// This is the O(N r) prediction of Sec. 2.3 (one read of the basis, one
// write per predicted state).  Each thread keeps one row of Us in registers
// and streams the output rows; coefficient columns are wave-uniform and come
// through the scalar cache.
#include <hip/hip_runtime.h>

#include "odmd_internal.h"
#include "pass.h"

namespace odmd {

template <typename TS, typename TO, int RB>
__global__ __launch_bounds__(256) void k_combine(CombineArgs c) {
  const DevState* __restrict__ st = c.st;
  const int pending = st->pending;
  const int ncols = pending ? st->rs : st->r;
  const int ue = pending && st->use_e;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= c.n) return;
  const TS* __restrict__ Us = static_cast<const TS*>(c.Us);
  const TS* __restrict__ Es = static_cast<const TS*>(c.Es);
  TO* __restrict__ out = static_cast<TO*>(c.out);
  double u[RB];
  const TS* __restrict__ T = Us + (i >> 6) * (int64_t)c.ct * 64 + (i & 63);
#pragma unroll
  for (int j = 0; j < RB; ++j) u[j] = j < ncols ? (double)T[j * 64] : 0.0;
  const double e = ue ? (double)Es[i] : 0.0;
  const int k0 = blockIdx.y * c.kb;
  const int k1 = min(c.K, k0 + c.kb);
  // coefficients are read-only for the launch: scalar loads via the
  // constant address space
  typedef const __attribute__((address_space(4))) double* cdp;
  cdp A = (cdp)st->coefA;
  cdp B = (cdp)st->coefB;
  for (int k = k0; k < k1; ++k) {
    asm volatile("" : "+s"(A), "+s"(B));
    double acc = e * B[k];
#pragma unroll
    for (int j = 0; j < RB; ++j) acc = __builtin_fma(u[j], A[k * RMAX + j], acc);
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
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_combine(const CombineArgs& c, int basis_f64, int out_f32, int rb, hipStream_t s) {
  if (basis_f64) return out_f32 ? launch_t<double, float>(c, rb, s) : launch_t<double, double>(c, rb, s);
  return out_f32 ? launch_t<float, float>(c, rb, s) : launch_t<float, double>(c, rb, s);
}

}  // namespace odmd
