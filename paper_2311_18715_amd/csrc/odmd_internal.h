// Internal layout shared by the HIP kernels and the host runtime.
//
// Per stream the device holds:
//   S         stored basis columns, in tiles of 64 rows (element (i, c) at
//             ((i/64)*ct + c)*64 + i%64, column-major inside a tile), ct
//             columns per tile, storage type TS (double or float);
//   partials  per-workgroup partial sums of the streaming pass;
//   DevState  the small FP64 state below.
//
// Brand's deferred form of the column append (the paper follows Brand's
// algorithm, Sec. 2.3): the logical basis U (the paper's L) is S[:, :m] Q with
// a small FP64 matrix Q (m x r).  An update stores its residual e as a new
// column of S and multiplies Q by the update's rotation; S itself is only
// rewritten (S[:, :r] <- S Q, Q <- I) when its ct columns are used up, by a
// streaming pass that does it on the way.  Most passes therefore read the
// basis once and write one column.
#pragma once
#include <stdint.h>

namespace odmd {

constexpr int RMAX = 64;          // rank cap
constexpr int MMAX = RMAX + 1;    // core size (r + 1)
constexpr int CMAX = 72;          // stored columns per tile, at most
constexpr int FOLD_SLACK = 16;    // pending stored columns (beyond r, or r_max for the capacity) before a refold
constexpr int PW = 2 * CMAX + 6;  // partial-sum record per workgroup
// Streaming-pass launch shape of a stream, fixed at creation (the
// partition sets the order of the pass's sums, so it never changes for a
// handle, batched or not):
//   wide (n >= PASS_WIDE_MIN_N): 512-thread workgroups, one per 256 rows, at
//        most 256 of them: one workgroup per CU for a stream that runs alone;
//   deep (smaller n): 256-thread workgroups, one per 512 rows, at most 512:
//        more 16-row units per wave, so that the one-unit-ahead prefetch
//        hides the load latency of short row ranges.
struct PassShape {
  int threads, rows_per_block, max_blocks;
};
constexpr PassShape PASS_WIDE = {512, 256, 256};
constexpr PassShape PASS_DEEP = {256, 512, 512};
constexpr int64_t PASS_WIDE_MIN_N = 131072;
// the built-in rule; a caller may give any valid shape instead (tuned ones)
inline PassShape default_shape(int64_t n) { return n >= PASS_WIDE_MIN_N ? PASS_WIDE : PASS_DEEP; }
// workgroup sizes the pass is compiled for, and the bounds a shape must keep
inline bool valid_shape(const PassShape& sh) {
  return (sh.threads == PASS_WIDE.threads || sh.threads == PASS_DEEP.threads) &&
         sh.rows_per_block >= 16 && sh.rows_per_block <= (1 << 24) && sh.rows_per_block % 16 == 0 &&
         sh.max_blocks >= 1 && sh.max_blocks <= 65536;
}
constexpr int CORE_THREADS = 1024;
constexpr int COEF_CHUNK = 512;   // prediction steps per coefficient chunk, at most
// The prediction's power-form coefficients c_k (rank r) of one chunk are
// kept in LDS with leading dimension r | 1: PC_LCOL doubles hold
// PC_LCOL / (r | 1) of them; the chunk size for that rank is that count
// rounded down to whole 16-state blocks of the read-out.
constexpr int PC_LCOL = 11264;
inline
#ifdef __HIPCC__
__host__ __device__
#endif
int coef_chunk(int r) {
  const int c = PC_LCOL / (r | 1) / 16 * 16;
  return c < COEF_CHUNK ? c : COEF_CHUNK;
}

// reduced partial-sum record layout (doubles)
constexpr int P_SUE = 0;             // S^T e         [0, CMAX)
constexpr int P_SUY = CMAX;          // S^T y         [CMAX, 2 CMAX)
constexpr int P_EE = 2 * CMAX;       // e . e
constexpr int P_EY = 2 * CMAX + 1;   // e . y
constexpr int P_XX = 2 * CMAX + 2;   // x . x
constexpr int P_YY = 2 * CMAX + 3;   // y . y
constexpr int P_XH = 2 * CMAX + 4;   // h . x  (row-hashed weights, see row_weight)
constexpr int P_YH = 2 * CMAX + 5;   // h . y

// latched status bits
constexpr int ST_NONFINITE = 1;
constexpr int ST_SEQ = 2;
constexpr int ST_NOCONV = 4;
constexpr int ST_EMPTY = 8;

struct DevState {
  // scalars (int block first, then doubles)
  int r;          // logical rank
  int m;          // stored columns in use (U = S[:, :m] Q), r <= m
  int refold;     // the next pass rewrites S[:, :r] = S Q (no free column left)
  int general;    // general pairs: B = Y W kept as B = T R (second state)
  int status;     // latched error bits
  int sweeps;     // Jacobi sweeps of the last core SVD
  int eig_valid;  // eigen cache belongs to the current model
  int eig_status; // 0 ok, else iteration cap hit
  long long m_acc;   // accepted pairs
  double tol;     // effective tolerance
  double yy_prev; // y.y of the last accepted pair (chaining fingerprint)
  double last_rho;
  double yh_prev; // h.y of the last accepted pair (second fingerprint)
  double pad_[3];
  // host-visible copy of `status` (a word of the handle's mapped pinned
  // memory), rewritten by every kernel that latches a bit, so that the host
  // can read the latched status of finished work without a device call
  unsigned* smirror;
  // vectors and matrices; r x r matrices column-major with leading dim RMAX
  double sigma[RMAX];
  double w[RMAX];
  double py[RMAX];      // U^T y_last: cached projection of the next x
  double a[CMAX];       // Q p1: coefficients of the next pass's first projection
  double p1[RMAX];      // U^T x of a general pair (chained pairs use py)
  double Q[RMAX * CMAX];      // m x r, row c (stored column c) at Q + c*RMAX
  double C[RMAX * RMAX];      // r x r: shifted product W[2:]^T W[:-1] (chained
                              // pairs) or G = U^T B (general pairs)
  double At[RMAX * RMAX];     // A~ (r x r)
  // eigen cache
  double lam_re[RMAX], lam_im[RMAX];
  double V_re[RMAX * RMAX], V_im[RMAX * RMAX];
  // read-out coefficients of one chunk: rows j < m, column k at coefA + k*CMAX
  double coefA[CMAX * COEF_CHUNK];
  double cfwd[RMAX];    // A~^k p_y at the end of the last prediction chunk
};

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

#ifdef __HIPCC__
// Weight of global row i in the chaining fingerprint h . x: a multiplicative
// hash of the index mapped to [1, 2) with 20 random bits (exact in FP64), so
// that a sign flip or a permutation of x changes h . x where x . x does not.
__device__ __forceinline__ double row_weight(int64_t i) {
  uint32_t k = (uint32_t)i * 2654435761u;
  k ^= k >> 15;
  k *= 2246822519u;
  k ^= k >> 13;
  return 1.0 + (double)(k >> 12) * 0x1p-20;
}

// Latch status bits (one thread) and mirror the result to the host word.
__device__ inline void latch_status(DevState* st, int bits) {
  st->status |= bits;
  if (st->smirror) *reinterpret_cast<volatile unsigned*>(st->smirror) = (unsigned)st->status;
}
#endif

// The live-column bucket of m stored columns (the pass is compiled for
// buckets 8, 16, ..., 72 and reads the first bucket >= m columns), as a
// batched pass chooses it on the device for a stream of capacity kb >= m.
inline
#ifdef __HIPCC__
__host__ __device__
#endif
int live_variant(int m, int kb) {
  const int b = m <= 8 ? 8 : (m + 7) / 8 * 8;
  return b < kb ? b : kb;
}

// stored-column capacity of a stream with rank cap r_max (multiple of 8)
inline int fold_capacity(int r_max) {
  const int c = (r_max + FOLD_SLACK + 7) / 8 * 8;
  return c < CMAX ? c : CMAX;
}

}  // namespace odmd
