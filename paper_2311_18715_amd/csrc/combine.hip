// Rollout / basis read-out: out[k] = U c_k for a block of coefficient
// columns, with U = S[:, :m] Q the logical basis (Q folded into the
// coefficients by the caller's coefficient kernel):
//     out[k*ldo + i] = sum_{j < m} S(i, j) * coefA[k*CMAX + j],
// S(i, j) stored at ((i/64)*ct + j)*64 + i%64 (64-row tiles).
// This is the O(N r) prediction of Sec. 2.3 (one read of the basis, one
// write per predicted state).
//
// As a product it is Out (K x n) = Coef (K x m) S^T (m x n) with a short
// contraction (m <= 72): 2 K n m flops against K n output writes.  For
// FP64 states the writes bound it (a 500-state read-out at n = 160,000 moves
// 889 MB, 178 us at the device-copy rate, against 98 us of FP64
// matrix-core time); for FP32 states and wide bases the two are close.  It
// runs on the FP64 matrix cores (16x16x4): a wavefront takes 16 rows of one tile in
// the streaming pass's operand layout (lane l holds row l%16 of stored
// columns 4 kk + l/16, so one column of the unit is a 128-byte line for
// FP64) and multiplies them by 16-step blocks of coefficients staged in LDS
// in the operand layout; lane l then holds states 4 v + l/16 of the block
// at row l%16, so 16 lanes write 16 consecutive rows of one state (streaming
// stores: the states are not read again here).  The
// stored values convert exactly to FP64, the coefficients are FP64 and so
// are the sums; the output is rounded once, to its type.  A workgroup covers
// a contiguous share of the rows (about CB_RPW or more: the grid holds no more
// workgroups than the GPU runs at once) and 16 NS states; the stored
// columns are read once per 16 NS states.  FP32 states from FP32 or BF16
// stored columns take k_combine32 instead (FP32 matrix cores, 128-byte
// stores); a few states (K <= 4) take k_combine_rows.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <map>
#include <mutex>
#include <utility>

#include "odmd_internal.h"
#include "pass.h"
#include "storage.h"

namespace odmd {

typedef double d4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float to_float_value(float v) { return v; }
__device__ __forceinline__ float to_float_value(bf16 v) { return __uint_as_float((uint32_t)v.bits << 16); }

constexpr int CB_THREADS = 256;          // four wavefronts
constexpr int CB_RPW = 512;              // rows per workgroup, at least

// NS 16-state blocks per workgroup (the host picks NS from the number of
// states, so that a short rollout computes no more than 16 states in vain)
template <typename TS, typename TO, int RB, int NS>
__global__ __launch_bounds__(CB_THREADS) void k_combine(CombineArgs c) {
  typedef Storage<TS> SC;
  constexpr int KK = RB / 4;                 // k-steps over the stored columns
  constexpr int NW = CB_THREADS / 64;
  const DevState* __restrict__ st = c.st;
  const int m = st->m;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, l16 = lane & 15;
  const int k0 = blockIdx.y * (16 * NS);

  // coefficients of the workgroup's states in the A-operand layout:
  // sC[s][kk][lane] = coef(state k0 + 16 s + lane%16, column 4 kk + lane/16)
  __shared__ double sC[NS][KK][64];
  for (int idx = threadIdx.x; idx < NS * KK * 64; idx += CB_THREADS) {
    const int ln = idx & 63, kk = (idx >> 6) % KK, s = (idx >> 6) / KK;
    const int k = k0 + 16 * s + (ln & 15), col = 4 * kk + (ln >> 4);
    sC[s][kk][ln] = (k < c.K && col < m) ? st->coefA[k * CMAX + col] : 0.0;
  }

  const TS* __restrict__ Us = static_cast<const TS*>(c.Us);
  TO* __restrict__ out = static_cast<TO*>(c.out);
  // the workgroup's rows: a contiguous share of the 16-row units (the
  // launch sizes the grid to the workgroups the GPU holds at once, so the
  // last round of workgroups does not run the chip part empty)
  const int64_t units = (c.n + 15) / 16;
  const int64_t ub = (int64_t)blockIdx.x * units / gridDim.x;
  const int64_t ue = (int64_t)(blockIdx.x + 1) * units / gridDim.x;
  const int64_t r0 = 16 * ub;
  const int nunit = (int)(ue - ub);
  const int kmax = (m + 3) / 4;              // live k-steps (uniform)
  // the unit's stored values stay in their storage type until used; the next
  // unit's loads are in flight while the current one is multiplied
  auto load = [&](int u, TS (&A)[KK]) {
    const int64_t row0 = r0 + 16 * u;        // 16-row units never straddle a tile
    const TS* __restrict__ T = Us + (row0 >> 6) * (int64_t)c.ct * 64 + (row0 & 63);
#pragma unroll
    for (int kk = 0; kk < KK; ++kk)
      if (kk < kmax) A[kk] = T[(4 * kk + q) * 64 + l16];
  };
  TS A[KK], An[KK];
  int u = wave;
  if (u < nunit) load(u, A);
  __syncthreads();
  for (; u < nunit; u += NW) {
    if (u + NW < nunit) load(u + NW, An);    // uniform
    d4_t d[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) d[s] = d4_t{0.0, 0.0, 0.0, 0.0};
    // the NS accumulator chains are independent: k-steps outermost
#pragma unroll
    for (int kk = 0; kk < KK; ++kk) {
      if (kk < kmax) {                       // uniform
        const double a = SC::to_double(A[kk]);
#pragma unroll
        for (int s = 0; s < NS; ++s)
          d[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(sC[s][kk][lane], a, d[s], 0, 0, 0);
      }
    }
    // the states are written once and not read again here: streaming stores
    const int64_t row = r0 + 16 * u + l16;
    if (row < c.n) {
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int k = k0 + 16 * s + 4 * v + q;
          if (k < c.K) __builtin_nontemporal_store((TO)d[s][v], out + (int64_t)k * c.ldo + row);
        }
    }
#pragma unroll
    for (int kk = 0; kk < KK; ++kk) A[kk] = An[kk];
  }
}

// FP32 states from FP32 or BF16 stored columns: the same product on the
// FP32 matrix cores (32x32x2, twice the FP64 rate), which also writes
// whole 128-byte lines: a wavefront takes 32 consecutive rows of one tile
// (lane l supplies row l%32 of stored column 2 kk + l/32; 32 lanes read a
// 128-byte line of a column), and register r of lane l holds state
// 8 (r/4) + 4 (l/32) + r%4 of a 32-state block at row l%32, so 32 lanes
// write 32 consecutive rows of one state.  The stored values are exact in
// FP32; the coefficients are rounded to FP32 and the sums are FP32 (about
// m FP32 roundings per state against one for the FP64 path: the output is
// FP32 either way).  NS 32-state blocks per workgroup; with one block the
// k-steps alternate between two accumulators, so that two product chains
// are in flight.
template <typename TS, int RB, int NS>
__global__ __launch_bounds__(CB_THREADS, 2) void k_combine32(CombineArgs c) {
  constexpr int KK = RB / 2;                 // k-steps over the stored columns
  constexpr int NA = NS == 1 ? 2 : 1;        // accumulators per block
  constexpr int NW = CB_THREADS / 64;
  typedef float f16v __attribute__((ext_vector_type(16)));
  const DevState* __restrict__ st = c.st;
  const int m = st->m;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int h = lane >> 5, l32 = lane & 31;
  const int k0 = blockIdx.y * (32 * NS);

  // sC[s][kk][lane] = coef(state k0 + 32 s + lane%32, column 2 kk + lane/32)
  __shared__ float sC[NS][KK][64];
  for (int idx = threadIdx.x; idx < NS * KK * 64; idx += CB_THREADS) {
    const int ln = idx & 63, kk = (idx >> 6) % KK, s = (idx >> 6) / KK;
    const int k = k0 + 32 * s + (ln & 31), col = 2 * kk + (ln >> 5);
    sC[s][kk][ln] = (k < c.K && col < m) ? (float)st->coefA[k * CMAX + col] : 0.f;
  }

  const TS* __restrict__ Us = static_cast<const TS*>(c.Us);
  float* __restrict__ out = static_cast<float*>(c.out);
  const int64_t units = (c.n + 31) / 32;     // 32-row units (two per 64-row tile)
  const int64_t ub = (int64_t)blockIdx.x * units / gridDim.x;
  const int64_t ue = (int64_t)(blockIdx.x + 1) * units / gridDim.x;
  const int64_t r0 = 32 * ub;
  const int nunit = (int)(ue - ub);
  const int kmax = (m + 1) / 2;              // live k-steps (uniform)
  auto load = [&](int u, float (&B)[KK]) {
    const int64_t row0 = r0 + 32 * u;
    const TS* __restrict__ T = Us + (row0 >> 6) * (int64_t)c.ct * 64 + (row0 & 63);
#pragma unroll
    for (int kk = 0; kk < KK; ++kk)
      if (kk < kmax) B[kk] = to_float_value(T[(2 * kk + h) * 64 + l32]);
  };
  float B[KK];
  __syncthreads();
  for (int u = wave; u < nunit; u += NW) {
    load(u, B);                              // two waves per SIMD hide the loads
    f16v d[NS][NA];
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int a = 0; a < NA; ++a) d[s][a] = f16v{};
#pragma unroll
    for (int kk = 0; kk < KK; ++kk) {
      if (kk < kmax) {                       // uniform
#pragma unroll
        for (int s = 0; s < NS; ++s)
          d[s][kk % NA] = __builtin_amdgcn_mfma_f32_32x32x2f32(sC[s][kk][lane], B[kk], d[s][kk % NA], 0, 0, 0);
      }
    }
    const int64_t row = r0 + 32 * u + l32;
    if (row < c.n) {
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        f16v e = d[s][0];
        if (NA == 2) e += d[s][NA - 1];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int k = k0 + 32 * s + 8 * (r >> 2) + 4 * h + (r & 3);
          if (k < c.K) __builtin_nontemporal_store(e[r], out + (int64_t)k * c.ldo + row);
        }
      }
    }
  }
}

// A few states (a one-step prediction, Sec. 2.3's u(t + dt)): bound by the
// read of the stored columns, not by the flops.  One row per lane (a wave
// reads 64 consecutive rows of a column, one 64-row tile), the coefficients
// of each state uniform across the wave (scalar loads); the stored values
// are read once for all the states of the launch.
constexpr int CR_KMAX = 4;
template <typename TS, typename TO, int RB>
__global__ __launch_bounds__(256) void k_combine_rows(CombineArgs c) {
  const DevState* __restrict__ st = c.st;
  const int m = st->m;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= c.n) return;
  const TS* __restrict__ T = static_cast<const TS*>(c.Us) + (i >> 6) * (int64_t)c.ct * 64 + (i & 63);
  double u[RB];
#pragma unroll
  for (int j = 0; j < RB; ++j) u[j] = j < m ? Storage<TS>::to_double(T[j * 64]) : 0.0;
  typedef const __attribute__((address_space(4))) double* cdp;
  cdp A = (cdp)st->coefA;
  TO* __restrict__ out = static_cast<TO*>(c.out);
  for (int k = 0; k < c.K; ++k) {
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < RB; ++j) acc = __builtin_fma(u[j], A[k * CMAX + j], acc);
    out[(int64_t)k * c.ldo + i] = (TO)acc;
  }
}

// Workgroups of kernel f the GPU holds at once (its occupancy per CU times
// the CUs of the current device), cached per kernel and device.
static int resident_blocks(const void* f) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find({f, dev});
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, CB_THREADS, 0) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return cache[{f, dev}] = per_cu * cus;
}

// Row workgroups: one per CB_RPW rows at most, and no more than the GPU holds
// at once together with the launch's other state blocks (then every
// workgroup gets a larger, equal share of the rows).  Workgroups go to the
// eight XCDs in turn by linear index x + g y; with g a multiple of 8 the
// state blocks of one row share run on the same XCD and read its stored
// columns through one L2 (with g = 170 and three state blocks, the columns
// were fetched three times).
template <typename K>
static dim3 combine_grid(K f, const CombineArgs& c, int NS) {
  const unsigned ys = (unsigned)((c.K + 16 * NS - 1) / (16 * NS));
  int64_t g = (c.n + CB_RPW - 1) / CB_RPW;
  const int res = resident_blocks(reinterpret_cast<const void*>(f));
  if (res > 0) g = std::min<int64_t>(g, std::max<int64_t>(1, res / (int64_t)ys));
  if (ys > 1 && g > 8) g = g / 8 * 8;
  return dim3((unsigned)g, ys);
}

template <typename TS, typename TO, int NS>
static hipError_t launch_ns(const CombineArgs& c, int rb, hipStream_t s) {
  const dim3 block(CB_THREADS);
  switch (rb) {
#define ODMD_CASE(RB) \
  case RB: hipLaunchKernelGGL((k_combine<TS, TO, RB, NS>), combine_grid(k_combine<TS, TO, RB, NS>, c, NS), \
                              block, 0, s, c); break;
    ODMD_CASE(8) ODMD_CASE(16) ODMD_CASE(24) ODMD_CASE(32) ODMD_CASE(40) ODMD_CASE(48)
    ODMD_CASE(56) ODMD_CASE(64) ODMD_CASE(72)
#undef ODMD_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename TS, int NS>
static hipError_t launch_ns32(const CombineArgs& c, int rb, hipStream_t s) {
  const dim3 block(CB_THREADS);
  switch (rb) {
#define ODMD_CASE(RB) \
  case RB: hipLaunchKernelGGL((k_combine32<TS, RB, NS>), combine_grid(k_combine32<TS, RB, NS>, c, 2 * NS), \
                              block, 0, s, c); break;
    ODMD_CASE(8) ODMD_CASE(16) ODMD_CASE(24) ODMD_CASE(32) ODMD_CASE(40) ODMD_CASE(48)
    ODMD_CASE(56) ODMD_CASE(64) ODMD_CASE(72)
#undef ODMD_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename TS, typename TO>
static hipError_t launch_rows(const CombineArgs& c, int rb, hipStream_t s) {
  const dim3 grid((unsigned)((c.n + 255) / 256)), block(256);
  switch (rb) {
#define ODMD_CASE(RB) \
  case RB: hipLaunchKernelGGL((k_combine_rows<TS, TO, RB>), grid, block, 0, s, c); break;
    ODMD_CASE(8) ODMD_CASE(16) ODMD_CASE(24) ODMD_CASE(32) ODMD_CASE(40) ODMD_CASE(48)
    ODMD_CASE(56) ODMD_CASE(64) ODMD_CASE(72)
#undef ODMD_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename TS, typename TO>
static hipError_t launch_t(const CombineArgs& c, int rb, hipStream_t s) {
  if (c.K <= CR_KMAX) return launch_rows<TS, TO>(c, rb, s);
  if constexpr (std::is_same<TO, float>::value && !std::is_same<TS, double>::value) {
    if (c.K <= 32) return launch_ns32<TS, 1>(c, rb, s);
    if (c.K <= 64) return launch_ns32<TS, 2>(c, rb, s);
    return launch_ns32<TS, 4>(c, rb, s);
  }
  // more 16-state blocks per workgroup: more independent accumulator
  // chains per wave (the FP64 matrix-core chains are latency-bound: 500
  // states at n = 160,000 and 56 columns took 182 us of matrix-core time
  // with eight blocks against 237 us with four) and fewer re-reads of the
  // stored columns, at the price of LDS (eight blocks of 72 columns: 72 KB)
  if (c.K <= 16) return launch_ns<TS, TO, 1>(c, rb, s);
  if (c.K <= 32) return launch_ns<TS, TO, 2>(c, rb, s);
  if (c.K <= 64) return launch_ns<TS, TO, 4>(c, rb, s);
  return launch_ns<TS, TO, 8>(c, rb, s);
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
