// Host-side declarations of the kernel launchers (one per .hip file).
#pragma once
#include <hip/hip_runtime.h>

#include "odmd_internal.h"

namespace odmd {

struct PassArgs {
  void* Us;             // stored basis S: 64-row tiles, column-major inside a tile
  const void* x;        // snapshot x_k (io type)
  const void* y;        // snapshot x_k+1 (io type)
  double* partials;     // nblk records (stride PW) of 2 rb + 6 values
  const DevState* st;
  int64_t n;
  int64_t units;        // (unused by the kernels; kept for the host)
  int nblk;             // workgroups
  int ct;               // column capacity of a basis tile (rank bucket of r_max)
  void* eout;           // general pairs: the stored residual e also written here
                        // as a contiguous n-vector of the io type (else null)
  int threads;          // workgroup size of the stream's launch shape
  int rows2;            // wide-row variant: with 512 threads, FP32 and BF16 storage
                        // read two rows per lane (fixed per stream, like its shape)
};

// basis: storage type (0 double, 1 float, 2 bf16; the odmd_dtype codes);
// rb: live-column bucket of the launch (multiple of 8, >= the stored
// columns in use m, <= the tile capacity ct).  e0 / e1 (may be null): events
// that take the kernel's own start and end timestamps.
hipError_t launch_pass(const PassArgs& p, int basis, int rb, hipStream_t s,
                       hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// Projection-only sweep of a general pair (same records with e = x: S^T x,
// S^T y, x.x, x.y, x.x, y.y; stores nothing, never refolds).
hipError_t launch_proj(const PassArgs& p, int basis, int rb, hipStream_t s);

// One stream of a batched pass launch (device-resident table, sorted by blk0).
struct PassDesc {
  void* Us;
  const void* x;
  const void* y;
  double* partials;
  const DevState* st;
  int64_t n;
  int nblk;             // workgroups of this stream
  int blk0;             // its first workgroup in the launch
  int ct;               // column capacity of its basis tiles
};
// threads: the launch shape's workgroup size, common to the streams of d
hipError_t launch_pass_batch(const PassDesc* d, int nd, int nblocks, int threads, int rows2, int basis,
                             int rb, hipStream_t s);
// The same, each workgroup running the live bucket of its stream's m, read
// on the device (live_variant; plans and graphs): one kernel per capacity
// kb of the streams of d; the core then takes rb = -kb.
hipError_t launch_pass_batch_live(const PassDesc* d, int nd, int nblocks, int threads, int rows2,
                                  int basis, int kb, hipStream_t s);

// Gram matrix of a BF16 basis after a refold (gram.hip): per-workgroup
// records of the 16x16 block pairs I <= J of the 64 columns
constexpr int GRAM_BLOCKS = RMAX / 16;
constexpr int GRAM_PAIRS = GRAM_BLOCKS * (GRAM_BLOCKS + 1) / 2;
constexpr int GRAM_REC = GRAM_PAIRS * 256;   // doubles per record
struct GramArgs {
  const DevState* st;
  const void* Us;       // BF16 stored columns (64-row tiles)
  double* rec;          // nwg records of GRAM_REC doubles
  int64_t n;
  int ct;               // column capacity of a tile
  int nwg;              // workgroups (records)
  int blk0;             // batched launch: the stream's first workgroup
};
// workgroups of the Gram kernel for n rows (one per 8192 rows, 1..64)
inline int gram_workgroups(int64_t n) {
  const int64_t w = (n + 8191) / 8192;
  return (int)(w < 1 ? 1 : (w > 64 ? 64 : w));
}
hipError_t launch_gram(const GramArgs& g, hipStream_t s);
hipError_t launch_gram_batch(const GramArgs* d, int nd, int nblocks, hipStream_t s);

struct CoreArgs {
  DevState* st;
  const double* partials;
  int nblk;
  int r_max;
  int jacobi_only;      // skip the secular solver (diagnostics)
  int rb;               // live-column bucket of the pass (compact partial records);
                        // -kb: the pass chose it on the device, live_variant(m, kb)
  int ct;               // stored-column capacity of the stream
  int fold_slack;       // refold once the stored columns reach r' + fold_slack
                        // (or the capacity); 0: only at the capacity
  unsigned* fb;         // host-visible word: (seq << 8) | stored columns after this update
  unsigned seq;         // update sequence number (24 bits) of this launch
  DevState* tst;        // general pairs: state of B = T R (R in its Q), else null
  const double* pt;     // general pairs: T sweep records, T^T e in the second half
  int rbt;              // general pairs: bucket of the T sweep
  const double* grec;   // BF16 basis: Gram records of the refolded columns (else null)
  int gnwg;             // their count
};

// General pairs, between the projection sweep and the streaming pass:
// reduces the projection records (S^T x) and sets p1 = U^T x = Q^T S^T x and
// the pass coefficients a = Q p1.
struct CoefArgs {
  DevState* st;
  const double* pproj;  // projection records (compact, 2 rb + 4 per workgroup)
  int nblk;
  int rb;               // bucket of the projection sweep
};
hipError_t launch_coef(const CoefArgs& c, hipStream_t s);
hipError_t launch_core(const CoreArgs& c, hipStream_t s, hipEvent_t e0 = nullptr,
                       hipEvent_t e1 = nullptr);
// one workgroup per entry of a device-resident CoreArgs table
hipError_t launch_core_batch(const CoreArgs* cs, int count, hipStream_t s);

struct CombineArgs {
  const DevState* st;   // coefficients coefA and the stored-column count m
  const void* Us;       // stored basis S (64-row tiles, column capacity ct)
  void* out;            // out[k*ldo + i], k < K
  int64_t n, ldo;
  int ct;               // column capacity of a basis tile
  int K;                // columns (predicted states) of this launch
};
// out type: 0 = FP64, 1 = FP32; basis: storage type code as for launch_pass
hipError_t launch_combine(const CombineArgs& c, int basis, int out_f32, int rb, hipStream_t s);

hipError_t launch_basis_coef(DevState* st, hipStream_t s);
// eigenvalues, and with vectors the unit eigenvectors V (cached per model)
hipError_t launch_eig(DevState* st, bool vectors, hipStream_t s);
// prediction coefficients of steps k0+1 .. k0+steps (steps <= coef_chunk(r_max))
// into columns koff .. koff+steps-1 of the read-out coefficients
hipError_t launch_power_coef(DevState* st, int k0, int steps, int koff, hipStream_t s);
// the first chunk of several streams: one workgroup per entry of
// device-resident tables of states and step counts
hipError_t launch_power_coef_batch(DevState* const* sts, const int* steps, int count, hipStream_t s);

}  // namespace odmd
