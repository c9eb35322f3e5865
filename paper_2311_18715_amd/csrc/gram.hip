// Gram matrix of a BF16 basis just rewritten by a refold.
//
// A refold rewrites S[:, :r] <- S Q (Brand's deferred rotation, Sec. 2.3's
// update held as stored columns times a small matrix) and rounds the new
// columns to BF16.  Their rounding (about 2^-9 of each entry) leaves the
// stored columns S' = fl(S Q) measurably non-orthogonal (||S'^T S' - I||_F
// about 1e-3), and the method's small problems assume an orthonormal basis.
// This kernel forms M = S'^T S' (FP64 sums of exact BF16 products), from
// which the small-state kernel takes the orthonormal basis S' M^-1/2 and
// carries the model over to it, before the update of that step.
//
// Layout: S' in 64-row tiles, column-major inside a tile, so four
// consecutive rows of a column are 8 contiguous bytes: exactly the operand
// of one lane of the 16x16x16 BF16 matrix-core product, which contracts over
// 16 rows.  A wavefront takes 16 rows of one tile (a unit) and, for every
// pair of 16-column blocks I <= J, adds S'_I^T S'_J of those rows (lane l
// supplies rows 4 (l/16) .. 4 (l/16) + 3 of column 16 I + l%16 for both
// operands); the FP32 block sums of a unit are added into FP64 accumulators.
// A workgroup sums its waves in a fixed order and writes one record per
// workgroup; the small-state kernel adds the records in index order, so the
// result is bitwise reproducible.  The kernel returns at once unless the
// pass of this update refolded (the host launches it after every pass of a
// BF16 stream; only the refold passes need it).
#include <hip/hip_runtime.h>

#include "odmd_internal.h"
#include "pass.h"

namespace odmd {

typedef short s4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

constexpr int GRAM_THREADS = 512;

__device__ __forceinline__ void gram_body(const GramArgs& g, int wg) {
  const DevState* __restrict__ st = g.st;
  if (!st->refold) return;                   // uniform: no refold in this update's pass
  const int r = st->r;
  const int nb = (r + 15) / 16;              // 16-column blocks of the refolded columns
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, l16 = lane & 15;
  constexpr int NW = GRAM_THREADS / 64;

  double acc[GRAM_PAIRS][4];
#pragma unroll
  for (int p = 0; p < GRAM_PAIRS; ++p)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[p][v] = 0.0;

  const int64_t units = (g.n + 15) / 16;
  const int64_t u0 = (int64_t)wg * units / g.nwg, u1 = (int64_t)(wg + 1) * units / g.nwg;
  const uint16_t* __restrict__ Us = static_cast<const uint16_t*>(g.Us);
  for (int64_t u = u0 + wave; u < u1; u += NW) {
    // rows of the last tile past n are zero (never written)
    const uint16_t* T = Us + (u >> 2) * (int64_t)g.ct * 64 + 16 * (u & 3) + 4 * q;
    s4_t op[GRAM_BLOCKS];
#pragma unroll
    for (int I = 0; I < GRAM_BLOCKS; ++I)
      op[I] = I < nb ? *reinterpret_cast<const s4_t*>(T + (16 * I + l16) * 64) : s4_t{0, 0, 0, 0};
    int p = 0;
#pragma unroll
    for (int I = 0; I < GRAM_BLOCKS; ++I)
#pragma unroll
      for (int J = I; J < GRAM_BLOCKS; ++J, ++p) {
        if (J < nb) {                        // uniform
          const f4_t d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(op[I], op[J], f4_t{0.f, 0.f, 0.f, 0.f},
                                                                  0, 0, 0);
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[p][v] += (double)d[v];
        }
      }
  }
  // waves in index order into one LDS record, then the record to memory:
  // entry p * 256 + 4 lane + v is the (4 (lane/16) + v, lane%16) element of
  // block pair p (I <= J, row-major over I then J)
  __shared__ double red[GRAM_REC];
  for (int w = 0; w < NW; ++w) {
    if (wave == w) {
#pragma unroll
      for (int p = 0; p < GRAM_PAIRS; ++p)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int e = p * 256 + 4 * lane + v;
          red[e] = (w == 0 ? 0.0 : red[e]) + acc[p][v];
        }
    }
    __syncthreads();
  }
  double* __restrict__ out = g.rec + (int64_t)wg * GRAM_REC;
  for (int e = threadIdx.x; e < GRAM_REC; e += GRAM_THREADS) out[e] = red[e];
}

__global__ __launch_bounds__(GRAM_THREADS) void k_gram(GramArgs g) { gram_body(g, blockIdx.x); }

// Many streams in one launch: workgroup b belongs to the stream whose
// range [blk0, blk0 + nwg) contains b (a device-resident table sorted by blk0).
__global__ __launch_bounds__(GRAM_THREADS) void k_gram_batch(const GramArgs* __restrict__ d, int nd) {
  const int b = blockIdx.x;
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].blk0 <= b) lo = mid;
    else hi = mid - 1;
  }
  const GramArgs g = d[lo];
  gram_body(g, b - g.blk0);
}

hipError_t launch_gram(const GramArgs& g, hipStream_t s) {
  hipLaunchKernelGGL(k_gram, dim3(g.nwg), dim3(GRAM_THREADS), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_gram_batch(const GramArgs* d, int nd, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_gram_batch, dim3(nblocks), dim3(GRAM_THREADS), 0, s, d, nd);
  return hipGetLastError();
}

}  // namespace odmd
