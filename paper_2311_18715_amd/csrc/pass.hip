// Kernels and launchers of the streaming pass with a fixed live-column
// bucket (the body, its layout and mapping: pass_body.h).
#include "pass_body.h"

namespace odmd {

template <typename TS, typename TIO, int RB, int NTH, bool R2>
__global__ __launch_bounds__(NTH) void k_pass(PassArgs p) {
  __shared__ double smem[pass_lds_doubles<RB, NTH>()];
  pass_body<TS, TIO, RB, NTH, R2>(p, blockIdx.x, smem);
}

template <typename TS, typename TIO, int RB, int NTH, bool R2>
__global__ __launch_bounds__(NTH) void k_proj(PassArgs p) {
  __shared__ double smem[pass_lds_doubles<RB, NTH>()];
  pass_body<TS, TIO, RB, NTH, R2, true>(p, blockIdx.x, smem);
}

template <typename TS, typename TIO, int RB, int NTH, bool R2>
__global__ __launch_bounds__(NTH) void k_pass_eout(PassArgs p) {
  __shared__ double smem[pass_lds_doubles<RB, NTH>()];
  pass_body<TS, TIO, RB, NTH, R2, false, true>(p, blockIdx.x, smem);
}

// Many streams of one storage type and live-column bucket in one launch: workgroup b
// belongs to the stream whose block range [blk0, blk0 + nblk) contains b, and
// runs exactly the work that workgroup b - blk0 of that stream's own launch
// would (same partition, same reduction order: results are bitwise equal).
template <typename TS, typename TIO, int RB, int NTH, bool R2>
__global__ __launch_bounds__(NTH) void k_pass_batch(const PassDesc* __restrict__ d, int nd) {
  typedef const __attribute__((address_space(4))) PassDesc* cdesc;
  cdesc D = (cdesc)d;
  const int b = blockIdx.x;
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (D[mid].blk0 <= b) lo = mid;
    else hi = mid - 1;
  }
  PassArgs p{};
  p.Us = D[lo].Us;
  p.x = D[lo].x;
  p.y = D[lo].y;
  p.partials = D[lo].partials;
  p.st = D[lo].st;
  p.n = D[lo].n;
  p.units = 0;
  p.nblk = D[lo].nblk;
  p.ct = D[lo].ct;
  __shared__ double smem[pass_lds_doubles<RB, NTH>()];
  pass_body<TS, TIO, RB, NTH, R2>(p, b - D[lo].blk0, smem);
}

// Launchers: storage type and live-column bucket select the instantiation,
// the stream's launch shape (PassShape::threads) the workgroup size, and its
// wide-row flag (512-thread FP32/BF16 streams only) the rows per lane.
template <typename TS, typename TIO, int RB>
static void batch_one(const PassDesc* d, int nd, int nblocks, int threads, int rows2, hipStream_t s) {
  constexpr int W = PASS_WIDE.threads, D = PASS_DEEP.threads;
  if constexpr (Storage<TS>::RPL > 1) {
    if (threads == W && rows2) {
      hipLaunchKernelGGL((k_pass_batch<TS, TIO, RB, W, true>), dim3(nblocks), dim3(W), 0, s, d, nd);
      return;
    }
  }
  if (threads == W)
    hipLaunchKernelGGL((k_pass_batch<TS, TIO, RB, W, false>), dim3(nblocks), dim3(W), 0, s, d, nd);
  else
    hipLaunchKernelGGL((k_pass_batch<TS, TIO, RB, D, false>), dim3(nblocks), dim3(D), 0, s, d, nd);
}

template <typename TS, typename TIO, int RB, int NTH, bool R2>
static void launch_kind(const PassArgs& p, bool proj, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const dim3 grid(p.nblk);
  if (proj) hipExtLaunchKernelGGL((k_proj<TS, TIO, RB, NTH, R2>), grid, dim3(NTH), 0, s, e0, e1, 0, p);
  else if (p.eout) hipExtLaunchKernelGGL((k_pass_eout<TS, TIO, RB, NTH, R2>), grid, dim3(NTH), 0, s, e0, e1, 0, p);
  else hipExtLaunchKernelGGL((k_pass<TS, TIO, RB, NTH, R2>), grid, dim3(NTH), 0, s, e0, e1, 0, p);
}

template <typename TS, typename TIO, int RB>
static void launch_one(const PassArgs& p, bool proj, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  constexpr int W = PASS_WIDE.threads, D = PASS_DEEP.threads;
  if constexpr (Storage<TS>::RPL > 1) {
    if (p.threads == W && p.rows2) {
      launch_kind<TS, TIO, RB, W, true>(p, proj, s, e0, e1);
      return;
    }
  }
  if (p.threads == W) launch_kind<TS, TIO, RB, W, false>(p, proj, s, e0, e1);
  else launch_kind<TS, TIO, RB, D, false>(p, proj, s, e0, e1);
}

#define ODMD_BUCKETS(CASE) CASE(8) CASE(16) CASE(24) CASE(32) CASE(40) CASE(48) CASE(56) CASE(64) CASE(72)

template <typename TS, typename TIO>
static hipError_t launch_batch_rb(const PassDesc* d, int nd, int nblocks, int threads, int rows2,
                                  int rb, hipStream_t s) {
  switch (rb) {
#define ODMD_CASE(RB) \
  case RB: batch_one<TS, TIO, RB>(d, nd, nblocks, threads, rows2, s); break;
    ODMD_BUCKETS(ODMD_CASE)
#undef ODMD_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pass_batch(const PassDesc* d, int nd, int nblocks, int threads, int rows2,
                             int basis, int rb, hipStream_t s) {
  switch (basis) {
    case 0: return launch_batch_rb<double, double>(d, nd, nblocks, threads, rows2, rb, s);
    case 1: return launch_batch_rb<float, float>(d, nd, nblocks, threads, rows2, rb, s);
    case 2: return launch_batch_rb<bf16, float>(d, nd, nblocks, threads, rows2, rb, s);
  }
  return hipErrorInvalidValue;
}

template <typename TS, typename TIO>
static hipError_t launch_rb(const PassArgs& p, int rb, bool proj, hipStream_t s, hipEvent_t e0,
                            hipEvent_t e1) {
  switch (rb) {
#define ODMD_CASE(RB) \
  case RB: launch_one<TS, TIO, RB>(p, proj, s, e0, e1); break;
    ODMD_BUCKETS(ODMD_CASE)
#undef ODMD_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

static hipError_t launch_any(const PassArgs& p, int basis, int rb, bool proj, hipStream_t s,
                             hipEvent_t e0, hipEvent_t e1) {
  switch (basis) {
    case 0: return launch_rb<double, double>(p, rb, proj, s, e0, e1);
    case 1: return launch_rb<float, float>(p, rb, proj, s, e0, e1);
    case 2: return launch_rb<bf16, float>(p, rb, proj, s, e0, e1);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_pass(const PassArgs& p, int basis, int rb, hipStream_t s, hipEvent_t e0,
                       hipEvent_t e1) {
  return launch_any(p, basis, rb, false, s, e0, e1);
}

hipError_t launch_proj(const PassArgs& p, int basis, int rb, hipStream_t s) {
  return launch_any(p, basis, rb, true, s, nullptr, nullptr);
}

}  // namespace odmd
