// Body of the streaming pass, shared by its kernels (fixed live-column
// bucket, and the batched kernels that choose the bucket on the device).
//
// The streaming pass of the online DMD update (HBM-bound: one read of the live
// stored columns, one column written; the stored columns are rewritten only
// on the refold passes).
//
// One update appends the pair (x, y) to the snapshot matrices (Sec. 2.3).
// Brand's column append needs the projection of x onto the basis and the
// residual direction.  With the basis held as U = S[:, :m] Q, this pass
// computes, in one sweep over the rows:
//   * the first Gram-Schmidt residual e = x - U p1 = x - S a (a = Q p1, p1
//     the cached projection U^T x, equal to the previous step's U^T y for
//     chained pairs), stored as column `slot` of S;
//   * per-workgroup partial sums of S^T e, S^T y, e.e, e.y, x.x and y.y, from
//     which the small-state kernel forms the second Gram-Schmidt projection
//     p2 = U^T e = Q^T S^T e and U^T y (CGS2);
//   * on a refold pass (the small-state kernel sets it once the stored
//     columns reach their limit: the capacity, or r + 16 pending columns for
//     FP64/FP32 storage), S[:, :r] <- S Q in place on the matrix cores, with
//     e then stored as column r.
// For general (unchained) pairs the same sweep also serves as the projection
// of x (k_proj: e = x, nothing stored), writes e contiguously for the next
// sweep, and, run on the stored columns T of B = Y W = T R with zero
// coefficients, appends y to T and forms T^T e.
//
// Layout and mapping (CDNA4): S is stored in tiles of 64 rows, each tile
// column-major (element (i, c) at ((i/64)*ct + c)*64 + i%64), so one column of
// a tile is 64 contiguous elements.  A wavefront processes 16 rows at a time
// in the operand layout of the 16x16x4 matrix-core instruction: lane l holds
// row l%16 of columns 4*kk + l/16, so that
//   * the refold S Q is a chain of MFMAs (Q staged in LDS in the operand
//     layout);
//   * e needs only an in-lane dot product plus two cross-lane additions;
//   * the projections accumulate in-lane across all rows a lane sees and are
//     reduced once per workgroup, in a fixed order (bitwise reproducible).
// The next unit's loads are issued before the current unit is processed.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <type_traits>

#include "odmd_internal.h"
#include "pass.h"
#include "storage.h"
#include "xlane.h"

namespace odmd {

// Coefficients that stay constant for a whole launch (written only by the
// small-state kernel) are read through the constant address space.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;

typedef double d4_t __attribute__((ext_vector_type(4)));

// The refold S[:, :r] <- S Q runs in FP64 on the matrix cores for every
// storage type: the stored values convert exactly, Q enters unrounded and the
// sums are FP64, so the only error of the new columns is their own rounding
// to the storage type.  (Rounding Q to FP32 for an FP32 product perturbs
// the basis inside its own span by FP32 roundoff at every refold; that loss
// of orthogonality compounds and needs a rank tolerance far above the
// storage's resolution to stay stable.)
struct RefoldMfma {
  typedef d4_t acc_t;
  __device__ static cptr<double> Q(const DevState* s) { return (cptr<double>)s->Q; }
  __device__ static acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // result element v of lane l sits in result row dsub(l, v), column l % 16
  __device__ static int dsub(int l, int v) { return 4 * v + (l >> 4); }
};

// PROJ: projection-only sweep of a general pair (e = x: the sums S^T x,
// S^T y, x.x, x.y; nothing is stored and no refold happens).  EOUT: the
// stored residual is also written to p.eout (general pairs).
// LDS of the pass body (doubles): the refold's Q in operand order, the
// coefficients a, and the per-wave records.  The kernel provides it, so that
// kernels holding several bodies share one buffer.
template <int RB, int NTH>
constexpr int pass_lds_doubles() {
  constexpr int KK = RB / 4, NT = ((RB < RMAX ? RB : RMAX) + 15) / 16;
  return KK * NT * 64 + 4 * KK + (NTH / 64) * (2 * RB + 6);
}

template <typename TS, typename TIO, int RB, int NTH, bool R2, bool PROJ = false, bool EOUT = false>
__device__ __forceinline__ void pass_body(const PassArgs& p, const int blk, double* smem) {
  typedef Storage<TS> SC;
  // rows per lane (one load per column): R2, the stream's wide-row variant
  // (see PassArgs::rows2), reads two (16 lanes then read a whole line of an
  // FP32 column, half a line of a BF16 one), else one
  constexpr int RPL = R2 ? SC::RPL : 1;
  // the loaded rows of one column, packed (8 or 4 bytes)
  typedef typename std::conditional<RPL * sizeof(TS) == 8, uint64_t, uint32_t>::type raw_t;
  constexpr int UR = 16 * RPL;            // rows per unit
  constexpr int UPT = 64 / UR;            // units per 64-row tile
  constexpr int KK = RB / 4;              // k-steps over the RB live stored columns
  constexpr int NT = ((RB < RMAX ? RB : RMAX) + 15) / 16;   // 16-column output blocks of a refold (r <= RMAX)
  constexpr int NWAVE = NTH / 64;           // waves of the workgroup
  typedef RefoldMfma::acc_t acc_t;

  const DevState* __restrict__ st = p.st;
  const int m = st->m, r = st->r, refold = PROJ ? 0 : st->refold;
  const int slot = refold ? r : m;        // the column that receives e
  TS* __restrict__ Us = static_cast<TS*>(p.Us);
  const TIO* __restrict__ X = static_cast<const TIO*>(p.x);
  const TIO* __restrict__ Y = static_cast<const TIO*>(p.y);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, l16 = lane & 15;

  double accE[KK], accY[KK], sEE = 0.0, sEY = 0.0, sXX = 0.0, sYY = 0.0, sXH = 0.0, sYH = 0.0;
#pragma unroll
  for (int kk = 0; kk < KK; ++kk) accE[kk] = accY[kk] = 0.0;

  const int64_t units = (p.n + UR - 1) / UR;
  const int64_t u0 = (int64_t)blk * units / p.nblk;
  const int64_t u1 = (int64_t)(blk + 1) * units / p.nblk;

  // Addressing: a unit is 16 RPL rows of one tile (lane row group l16 holds
  // its rows RPL l16 .. RPL l16 + RPL - 1, read with one load per column:
  // for FP64 and FP32 storage 16 lanes read a whole 128-byte line of a
  // column), so its base is wave-uniform (scalar registers) and each lane adds a constant
  // 32-bit offset.  Rows of the last tile past n are never written and stay
  // zero, so stored columns are read without a row test.  Every load is
  // issued unconditionally, so the number in flight is fixed and the waits
  // can leave the prefetched unit outstanding: a k-step past the m live
  // columns re-reads k-step 0 (a cache hit) and meets zero coefficients (a
  // and the staged Q vanish past m; every stored value is finite, see the
  // residual store), x and y are read at a clamped row and zeroed past n.
  const uint32_t loff = (uint32_t)((q * 64 + RPL * l16) * sizeof(TS));
  typedef gbytes gbase_t;
  auto unit_base = [&](int64_t uu) -> gbase_t {
    const int64_t tile = uu / UPT;
    const uint64_t b = reinterpret_cast<uint64_t>(Us + tile * (int64_t)p.ct * 64 + UR * (uu % UPT));
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return (gbase_t)(((uint64_t)hi << 32) | lo);
  };
  auto load_unit = [&](int64_t uu, raw_t (&A)[KK], double (&xv)[RPL], double (&yv)[RPL]) {
    const gbase_t base = unit_base(uu);
#pragma unroll
    for (int kk = 0; kk < KK; ++kk) {
      const int ks = 4 * kk < m ? kk : 0;   // uniform
      if constexpr (RPL == SC::RPL) A[kk] = (raw_t)SC::rows(base + ks * 256 * (int)sizeof(TS) + loff);
      else A[kk] = (raw_t)SC::row(base + ks * 256 * (int)sizeof(TS) + loff);
    }
    const int64_t row0 = (uu / UPT) * 64 + UR * (uu % UPT) + RPL * l16;
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
      const int64_t rc = row0 + j < p.n ? row0 + j : p.n - 1;
      xv[j] = (double)X[rc];   // zeroed past n at the point of use
      yv[j] = (double)Y[rc];
    }
  };

  // software pipeline: the next unit's loads (the current unit's again on
  // the last round, so the count never varies) are in flight while the
  // current one is processed
  raw_t A[KK], An[KK];                    // RPL stored values per k-step, packed
  double xv[RPL], yv[RPL], xn[RPL], yn[RPL];
  // the coefficients a of the first projection go to LDS, with Q
  // pre-arranged in the MFMA operand layout (entry [kk][nt][lane] =
  // Q[4 kk + lane/16][16 nt + lane%16]) for a refold.  a is loaded before
  // the first unit, so that waiting for it leaves the unit's loads in flight.
  static_assert(NTH >= 4 * KK, "one thread per coefficient");
  double (*sG)[NT][64] = reinterpret_cast<double (*)[NT][64]>(smem);
  double* sa = smem + KK * NT * 64;      // a, zero past the m stored columns
  const int ca = threadIdx.x;
  const double a_c = (ca < 4 * KK && ca < m) ? st->a[ca] : 0.0;
  // (unconditional, as in the loop: a wave without a unit of its own
  // re-reads unit u0, which is in range, u0 < units, for every workgroup,
  // also one that gets no unit at all: with 32-row units there can be
  // fewer units than workgroups, u0 == u1 there, and its loop is empty)
  int64_t u = u0 + __builtin_amdgcn_readfirstlane(wave);
  load_unit(u < u1 ? u : u0, A, xv, yv);
  if (ca < 4 * KK) sa[ca] = a_c;
  if (refold) {
    cptr<double> Q = RefoldMfma::Q(st);
    for (int idx = threadIdx.x; idx < KK * NT * 64; idx += NTH) {
      const int ln = idx & 63, nt = (idx >> 6) % NT, kk = (idx >> 6) / NT;
      const int c = 4 * kk + (ln >> 4), col = 16 * nt + (ln & 15);
      sG[kk][nt][ln] = (c < m && col < r) ? Q[c * RMAX + col] : 0.0;
    }
  }
  __syncthreads();

  // (an empty asm statement that claims to change the packed values keeps
  // the compiler from holding every unpacked row live between the steps:
  // each step unpacks again)
  auto fence_rows = [&](raw_t (&V)[KK]) {
    if constexpr (RPL > 1) {
#pragma unroll
      for (int kk = 0; kk < KK; ++kk) asm volatile("" : "+v"(V[kk]));
    }
  };
  for (; u < u1; u += NWAVE) {
    const bool more = u + NWAVE < u1;
    load_unit(more ? u + NWAVE : u, An, xn, yn);
    const int64_t tile = u / UPT;
    const int rr0 = UR * (int)(u % UPT) + RPL * l16;   // the lane's first row in the tile
    const int64_t row0 = tile * 64 + rr0;
    TS* __restrict__ T = Us + tile * (int64_t)p.ct * 64;
#pragma unroll
    for (int j = 0; j < RPL; ++j)
      if (row0 + j >= p.n) xv[j] = yv[j] = 0.0;

    // e = x - S a, in FP64, stored as column `slot`
    double ed[RPL];
#pragma unroll
    for (int j = 0; j < RPL; ++j) ed[j] = xv[j];
    if constexpr (!PROJ) {
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        double s = 0.0;
#pragma unroll
        for (int kk = 0; kk < KK; ++kk)
          s = __builtin_fma(SC::to_double(SC::elem(A[kk], j)), sa[4 * kk + q], s);
        s = add_half_pair(add_row_pair(s));
        const TS es = SC::from_double(xv[j] - s);
        ed[j] = SC::to_double(es);    // the stored value, which the sums see
        // a non-finite residual (rejected by the small-state kernel, which
        // sees it in the sums below) is stored as zero: stored columns stay
        // finite
        if (q == 0 && row0 + j < p.n)
          T[slot * 64 + rr0 + j] = __builtin_isfinite(ed[j]) ? es : SC::from_double(0.0);
        if constexpr (EOUT) {
          if (q == 0 && row0 + j < p.n) static_cast<TIO*>(p.eout)[row0 + j] = (TIO)ed[j];
        }
      }
      fence_rows(A);
    }

    // projections, accumulated in-lane (the lane's rows in order)
#pragma unroll
    for (int kk = 0; kk < KK; ++kk) {
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        const double av = SC::to_double(SC::elem(A[kk], j));
        accE[kk] = __builtin_fma(av, ed[j], accE[kk]);
        accY[kk] = __builtin_fma(av, yv[j], accY[kk]);
      }
    }
    if (q == 0) {
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        const double hw = row_weight(row0 + j);
        sEE = __builtin_fma(ed[j], ed[j], sEE);
        sEY = __builtin_fma(ed[j], yv[j], sEY);
        sXX = __builtin_fma(xv[j], xv[j], sXX);
        sYY = __builtin_fma(yv[j], yv[j], sYY);
        sXH = __builtin_fma(hw, xv[j], sXH);
        sYH = __builtin_fma(hw, yv[j], sYH);
      }
    }

    // refold on the matrix cores, computed transposed: (S Q)^T = Q^T S^T, so
    // that lane l owns the rows of row group l%16 of S Q (one product chain
    // per row of the group); k-steps outermost keeps the NT accumulator
    // chains independent
    if (refold) {
      fence_rows(A);
      // one 16-column output block at a time keeps the accumulator small
      // (the refold pass is the rare one; the register budget is set for
      // the plain pass)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        if (16 * nt >= r) break;   // uniform: output blocks past the rank hold no column
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
          // the FP64 operands are converted again for every block and row,
          // not held across them (that would double the stored values'
          // registers)
          fence_rows(A);
          acc_t d = acc_t{0, 0, 0, 0};
#pragma unroll
          for (int kk = 0; kk < KK; ++kk)
            d = RefoldMfma::mma(sG[kk][nt][lane], SC::to_double(SC::elem(A[kk], j)), d);
          if (row0 + j < p.n) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int col = 16 * nt + RefoldMfma::dsub(lane, v);
              if (col < r) T[col * 64 + rr0 + j] = SC::from_double(d[v]);
            }
          }
        }
      }
    }
#pragma unroll
    for (int kk = 0; kk < KK; ++kk) A[kk] = An[kk];
#pragma unroll
    for (int j = 0; j < RPL; ++j) {
      xv[j] = xn[j];
      yv[j] = yn[j];
    }
  }

  // fixed-order reduction: across the 16 lanes that share a column (one
  // 16-lane row), then across the workgroup's waves in index order
#pragma unroll
  for (int kk = 0; kk < KK; ++kk) {
    accE[kk] = row_sum(accE[kk]);
    accY[kk] = row_sum(accY[kk]);
  }
  // the four scalar sums live in the first row only
  sEE = row_sum(sEE);
  sEY = row_sum(sEY);
  sXX = row_sum(sXX);
  sYY = row_sum(sYY);
  sXH = row_sum(sXH);
  sYH = row_sum(sYH);
  // record: [S^T e (RB) | S^T y (RB) | e.e e.y x.x y.y h.x h.y]
  double (*red)[2 * RB + 6] = reinterpret_cast<double (*)[2 * RB + 6]>(sa + 4 * KK);
  if (l16 == 0) {
#pragma unroll
    for (int kk = 0; kk < KK; ++kk) {
      red[wave][4 * kk + q] = accE[kk];
      red[wave][RB + 4 * kk + q] = accY[kk];
    }
  }
  if (lane == 0) {
    red[wave][2 * RB + 0] = sEE;
    red[wave][2 * RB + 1] = sEY;
    red[wave][2 * RB + 2] = sXX;
    red[wave][2 * RB + 3] = sYY;
    red[wave][2 * RB + 4] = sXH;
    red[wave][2 * RB + 5] = sYH;
  }
  __syncthreads();
  double* __restrict__ out = p.partials + (int64_t)blk * PW;
  for (int idx = threadIdx.x; idx < 2 * RB + 6; idx += NTH) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NWAVE; ++w) t += red[w][idx];
    out[idx] = t;
  }
}

}  // namespace odmd
