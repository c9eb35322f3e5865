// Streaming pass of the online DMD update (HBM-bound, one read of the basis).
//
// One update appends the pair (x, y) to the snapshot matrices (Sec. 2.3).
// Brand's column append needs the projection of x onto the basis and the
// residual direction; this pass computes, in one sweep over the rows:
//   * the pending rotation of the previous update, U = Us G + Es g^T,
//     written back to Us (so the basis is read once and written once);
//   * the first Gram-Schmidt residual e = x - U p1 with the cached
//     projection p1 = U^T x (equal to the previous step's U^T y for chained
//     pairs), stored to Es;
//   * per-workgroup partial sums of Us^T e, Es.e, e.e, x.x and of Us^T y,
//     Es.y, e.y, y.y.  The small-state kernel turns them into the second
//     Gram-Schmidt projection p2 = U^T e = G^T (Us^T e) + g (Es.e) and into
//     U^T y the same way, which completes the CGS2 step.
// Partial sums are reduced in a fixed order (wave reduce-scatter, then the
// workgroup's waves in index order) so results do not depend on timing.
#include <hip/hip_runtime.h>

#include "odmd_internal.h"
#include "pass.h"

namespace odmd {

template <int N, int O>
__device__ __forceinline__ void rs_step(double* v, int lane) {
  const bool up = (lane & O) != 0;
#pragma unroll
  for (int t = 0; t < N / 2; ++t) {
    const double keep = up ? v[t + N / 2] : v[t];
    const double send = up ? v[t] : v[t + N / 2];
    v[t] = keep + __shfl_xor(send, O, 64);
  }
}

// Recursive-halving reduce-scatter over a 64-wide wavefront: afterwards lane
// l holds in v[0 .. N/64) the wave sums of the entries [l*N/64, (l+1)*N/64).
template <int N>
__device__ __forceinline__ void wave_reduce_scatter(double* v, int lane) {
  static_assert(N % 64 == 0, "N must be a multiple of 64");
  rs_step<N, 32>(v, lane);
  rs_step<N / 2, 16>(v, lane);
  rs_step<N / 4, 8>(v, lane);
  rs_step<N / 8, 4>(v, lane);
  rs_step<N / 16, 2>(v, lane);
  rs_step<N / 32, 1>(v, lane);
}

// Coefficients that stay constant for a whole launch (written only by the
// small-state kernel) are read through the constant address space, so that
// wave-uniform reads become scalar loads broadcast to all lanes.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;

template <typename T> struct Rot;
template <> struct Rot<double> {
  __device__ static cptr<double> G(const DevState* s) { return (cptr<double>)s->G; }
  __device__ static cptr<double> g(const DevState* s) { return (cptr<double>)s->g; }
};
template <> struct Rot<float> {
  __device__ static cptr<float> G(const DevState* s) { return (cptr<float>)s->G32; }
  __device__ static cptr<float> g(const DevState* s) { return (cptr<float>)s->g32; }
};

__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Partial-record slot of entry g of group A (e products) or B (y products).
template <int RB>
__device__ __forceinline__ int slot_of(int idx, int NA) {
  const bool b = idx >= NA;
  const int g = b ? idx - NA : idx;
  if (g < RB) return (b ? P_SUY : P_SUE) + g;
  if (g == RB) return b ? P_SEY : P_SEE;
  if (g == RB + 1) return b ? P_EY : P_EE;
  if (g == RB + 2) return b ? P_YY : P_XX;
  return -1;
}

template <typename TS, typename TIO, int RB>
__device__ __forceinline__ void pass_body(const PassArgs& p, const DevState* __restrict__ st,
                                          int rs, int r, int pending, int use_e) {
  constexpr int NA = 64 * ((RB + 3 + 63) / 64);
  constexpr int KA = NA / 64;
  constexpr int NWAVE = PASS_THREADS / 64;
  TS* __restrict__ Us = static_cast<TS*>(p.Us);
  TS* __restrict__ Es = static_cast<TS*>(p.Es);
  const TIO* __restrict__ X = static_cast<const TIO*>(p.x);
  const TIO* __restrict__ Y = static_cast<const TIO*>(p.y);
  cptr<double> a = (cptr<double>)st->a;
  cptr<TS> G = Rot<TS>::G(st);
  cptr<TS> gv = Rot<TS>::g(st);
  const double beta = st->beta;
  const int64_t ld = p.ld;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;

  double accA[KA], accB[KA];
#pragma unroll
  for (int q = 0; q < KA; ++q) accA[q] = accB[q] = 0.0;

  const int t0 = (int)((int64_t)blockIdx.x * p.tiles / p.nblk);
  const int t1 = (int)((int64_t)(blockIdx.x + 1) * p.tiles / p.nblk);
  for (int tile = t0; tile < t1; ++tile) {
    // Keep the loop-invariant coefficient loads inside the loop: hoisted, the
    // r x r rotation would not fit in scalar registers and would spill.
    asm volatile("" : "+s"(G), "+s"(gv), "+s"(a));
    const int64_t i = (int64_t)tile * PASS_THREADS + threadIdx.x;
    const bool in = i < p.n;
    TS us[RB];
#pragma unroll
    for (int j = 0; j < RB; ++j) us[j] = (in && j < rs) ? Us[j * ld + i] : TS(0);
    const double es = (in && use_e) ? (double)Es[i] : 0.0;
    const double xi = in ? (double)X[i] : 0.0;
    const double yi = in ? (double)Y[i] : 0.0;

    // first Gram-Schmidt residual against the (rotated) basis, in FP64
    double e = xi;
#pragma unroll
    for (int j = 0; j < RB; ++j) e = fmad(-(double)us[j], a[j], e);
    e = fmad(-es, beta, e);
    const TS e_s = (TS)e;
    if (in) Es[i] = e_s;
    const double ed = (double)e_s;

    double v[NA];
#pragma unroll
    for (int j = 0; j < NA; ++j) v[j] = 0.0;
#pragma unroll
    for (int j = 0; j < RB; ++j) v[j] = (double)us[j] * ed;
    v[RB] = es * ed;
    v[RB + 1] = ed * ed;
    v[RB + 2] = xi * xi;
    wave_reduce_scatter<NA>(v, lane);
#pragma unroll
    for (int q = 0; q < KA; ++q) accA[q] += v[q];

#pragma unroll
    for (int j = 0; j < NA; ++j) v[j] = 0.0;
#pragma unroll
    for (int j = 0; j < RB; ++j) v[j] = (double)us[j] * yi;
    v[RB] = es * yi;
    v[RB + 1] = ed * yi;
    v[RB + 2] = yi * yi;
    wave_reduce_scatter<NA>(v, lane);
#pragma unroll
    for (int q = 0; q < KA; ++q) accB[q] += v[q];

    // pending rotation of the previous update: U = Us G + Es g^T
    if (pending) {
      const TS est = (TS)es;
#pragma unroll
      for (int k = 0; k < RB; ++k) {
        TS acc = est * gv[k];
#pragma unroll
        for (int j = 0; j < RB; ++j) acc = fmad(us[j], G[k * RMAX + j], acc);
        if (in && k < r) Us[k * ld + i] = acc;
      }
    }
  }

  __shared__ double red[NWAVE][2 * 128];
#pragma unroll
  for (int q = 0; q < KA; ++q) {
    red[wave][lane * KA + q] = accA[q];
    red[wave][NA + lane * KA + q] = accB[q];
  }
  __syncthreads();
  double* __restrict__ out = p.partials + (int64_t)blockIdx.x * PW;
  for (int idx = threadIdx.x; idx < 2 * NA; idx += PASS_THREADS) {
    const int s = slot_of<RB>(idx, NA);
    if (s < 0) continue;
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NWAVE; ++w) t += red[w][idx];
    out[s] = t;
  }
}

template <typename TS, typename TIO, int RB>
__global__ __launch_bounds__(PASS_THREADS) void k_pass(PassArgs p) {
  const DevState* __restrict__ st = p.st;
  pass_body<TS, TIO, RB>(p, st, st->rs, st->r, st->pending, st->use_e);
}

template <typename TS, typename TIO>
static hipError_t launch_rb(const PassArgs& p, int rb, hipStream_t s) {
  const dim3 grid(p.nblk), block(PASS_THREADS);
  switch (rb) {
    case 8: hipLaunchKernelGGL((k_pass<TS, TIO, 8>), grid, block, 0, s, p); break;
    case 16: hipLaunchKernelGGL((k_pass<TS, TIO, 16>), grid, block, 0, s, p); break;
    case 24: hipLaunchKernelGGL((k_pass<TS, TIO, 24>), grid, block, 0, s, p); break;
    case 32: hipLaunchKernelGGL((k_pass<TS, TIO, 32>), grid, block, 0, s, p); break;
    case 40: hipLaunchKernelGGL((k_pass<TS, TIO, 40>), grid, block, 0, s, p); break;
    case 48: hipLaunchKernelGGL((k_pass<TS, TIO, 48>), grid, block, 0, s, p); break;
    case 56: hipLaunchKernelGGL((k_pass<TS, TIO, 56>), grid, block, 0, s, p); break;
    case 64: hipLaunchKernelGGL((k_pass<TS, TIO, 64>), grid, block, 0, s, p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pass(const PassArgs& p, int basis_f64, int rb, hipStream_t s) {
  return basis_f64 ? launch_rb<double, double>(p, rb, s) : launch_rb<float, float>(p, rb, s);
}

}  // namespace odmd
