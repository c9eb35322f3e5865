// Batched streaming pass whose live-column bucket is chosen on the device.
//
// A plan (and a graph captured from it) cannot follow the stored-column
// count m from the host, so its passes were sized for each stream's full
// capacity KB, paying KB/4 k-steps per unit whatever m is.  Here each
// workgroup reads its stream's m and runs the instantiation of m's bucket
// (live_variant: the bucket a launch sized by the host's exact count picks;
// any bucket >= m gives the same bits, dead k-steps meeting zero
// coefficients), so results equal odmd_update_batch's.  The core derives
// the record length the pass wrote from the same m.  One kernel per
// capacity KB holds the buckets up to KB: its register count is the KB
// variant's (as when every pass ran at KB), and the buckets share the KB
// variant's LDS.
#include "pass_body.h"

namespace odmd {

template <typename TS, typename TIO, int NTH, bool R2, int KB>
__global__ __launch_bounds__(NTH) void k_pass_batch_live(const PassDesc* __restrict__ d, int nd) {
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
  const int blk = b - D[lo].blk0;
  __shared__ double smem[pass_lds_doubles<KB, NTH>()];   // shared by the variants
  const int rb = live_variant(p.st->m, KB);   // uniform
  switch (rb) {
#define ODMD_LIVE(B) \
  case B:                                                   \
    if constexpr (B <= KB) pass_body<TS, TIO, B, NTH, R2>(p, blk, smem); \
    break;
    ODMD_LIVE(8) ODMD_LIVE(16) ODMD_LIVE(24) ODMD_LIVE(32) ODMD_LIVE(40) ODMD_LIVE(48)
    ODMD_LIVE(56) ODMD_LIVE(64) ODMD_LIVE(72)
#undef ODMD_LIVE
    default: break;
  }
}

template <typename TS, typename TIO, int KB>
static void live_shape(const PassDesc* d, int nd, int nblocks, int threads, int rows2, hipStream_t s) {
  constexpr int W = PASS_WIDE.threads, DP = PASS_DEEP.threads;
  if constexpr (Storage<TS>::RPL > 1) {
    if (threads == W && rows2) {
      hipLaunchKernelGGL((k_pass_batch_live<TS, TIO, W, true, KB>), dim3(nblocks), dim3(W), 0, s, d, nd);
      return;
    }
  }
  if (threads == W)
    hipLaunchKernelGGL((k_pass_batch_live<TS, TIO, W, false, KB>), dim3(nblocks), dim3(W), 0, s, d, nd);
  else
    hipLaunchKernelGGL((k_pass_batch_live<TS, TIO, DP, false, KB>), dim3(nblocks), dim3(DP), 0, s, d, nd);
}

template <typename TS, typename TIO>
static hipError_t live_kb(const PassDesc* d, int nd, int nblocks, int threads, int rows2, int kb,
                          hipStream_t s) {
  switch (kb) {
#define ODMD_CASE(KB) \
  case KB: live_shape<TS, TIO, KB>(d, nd, nblocks, threads, rows2, s); break;
    ODMD_CASE(24) ODMD_CASE(32) ODMD_CASE(40) ODMD_CASE(48) ODMD_CASE(56) ODMD_CASE(64) ODMD_CASE(72)
#undef ODMD_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pass_batch_live(const PassDesc* d, int nd, int nblocks, int threads, int rows2,
                                  int basis, int kb, hipStream_t s) {
  switch (basis) {
    case 0: return live_kb<double, double>(d, nd, nblocks, threads, rows2, kb, s);
    case 1: return live_kb<float, float>(d, nd, nblocks, threads, rows2, kb, s);
    case 2: return live_kb<bf16, float>(d, nd, nblocks, threads, rows2, kb, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace odmd
