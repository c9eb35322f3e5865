/*
 * odmd.h -- online dynamic mode decomposition on one MI355X (gfx950).
 *
 * The library keeps, per snapshot stream, the online DMD of Sec. 2.3 of
 * "Accelerating Flow Simulations using Online Dynamic Mode Decomposition"
 * (arXiv 2311.18715): the truncated SVD U- = L S R^* of the input snapshot
 * matrix, updated by one rank-1 column append per time step (Brand's
 * incremental SVD, the paper's reference [brand2006fast]); the reduced
 * operator A~ = L^* U+ R S^-1; its eigendecomposition A~ = V Lambda V^-1;
 * and the prediction u(t) = Phi Lambda^(t/dt) Phi^+ u(0) with Phi = L V.
 *
 * Symbols used below: n is the state dimension (the paper's N), r the
 * current rank, r_max its cap, U the n x r left basis (the paper's L),
 * sigma the singular values, A~ the r x r reduced operator.
 *
 * Conventions for every call:
 *   - Every call returns an odmd_status; nothing aborts the process.
 *   - Arguments are checked on the host before any device work; a bad
 *     argument returns ODMD_EINVAL and leaves the handle untouched.
 *   - Pointers marked "device" must point to device memory of the GPU the
 *     handle was created on; "host" pointers to ordinary host memory.
 *   - Work is queued on the handle's HIP stream and returns before the GPU
 *     finishes, unless the call is marked (synchronising).  Errors that the
 *     GPU detects (non-finite input, unchained pair, no convergence) are
 *     latched in the handle and returned, then cleared, by the next
 *     synchronising call.
 *   - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef ODMD_H
#define ODMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct odmd_s* odmd_t;

/* Element types.  ODMD_F64 / ODMD_F32 may be used for the basis and for
 * snapshots; ODMD_BF16 only for the basis (with FP32 snapshots). */
typedef enum { ODMD_F64 = 0, ODMD_F32 = 1, ODMD_BF16 = 2 } odmd_dtype;

typedef enum {
  ODMD_OK = 0,
  ODMD_EINVAL = 1,     /* bad argument (checked on the host)              */
  ODMD_ENOMEM = 2,     /* device allocation failed / workspace too small  */
  ODMD_EEMPTY = 3,     /* eigs or predict on a rank-0 model               */
  ODMD_ENONFINITE = 4, /* a snapshot held NaN/Inf; that update was skipped */
  ODMD_ENOCONV = 5,    /* small SVD or eigen-iteration hit its sweep cap   */
  ODMD_ESEQ = 6,       /* x_k was not the previous x_k+1; update skipped   */
  ODMD_EDEVICE = 7     /* HIP runtime error or no usable device            */
} odmd_status;

/* Largest supported rank cap (the small FP64 problems live in one
 * workgroup's LDS). */
#define ODMD_RMAX 64

/*
 * Create a stream model with an FP64 basis and FP64 snapshots on the
 * current device's null stream; the library allocates its own device
 * memory.  n >= 1, 1 <= r_max <= min(n, ODMD_RMAX), 0 <= tol < 1.
 * tol is relative and serves both tests of the method's rank choice
 * (Sec. 2.3 leaves it open): a new direction is kept only if its residual
 * norm exceeds tol * ||x_k||, and after each update only singular values
 * above tol * sigma_1 are kept (at most r_max of them).
 * On success *h receives the handle (host pointer to a host handle).
 */
odmd_status odmd_create(int64_t n, int32_t r_max, double tol, odmd_t* h);

/*
 * As odmd_create, with the basis storage type, the snapshot (and
 * prediction output) type, the HIP stream (hipStream_t, NULL = null
 * stream) and optionally caller-owned device memory.
 *   basis: ODMD_F64, ODMD_F32 or ODMD_BF16 (stored columns rounded to
 *          nearest even; residuals, projections, the rotation of the stored
 *          columns and the small problems stay FP64; a BF16 basis is
 *          re-orthonormalised from the Gram matrix of its columns after
 *          each rewrite).  The effective tolerance is tol for FP64 and FP32
 *          bases and max(tol, 2^-12) for BF16: the rounding of a rewritten
 *          BF16 basis shows in the next snapshots as residuals of about
 *          2^-9 of their norm, which that tolerance truncates again.
 *   io:    ODMD_F64 or ODMD_F32; equal to basis for F64/F32 bases, ODMD_F32
 *          for a BF16 basis.
 *   The small SVD of each update is solved through its secular equation,
 *   with one-sided Jacobi as the fallback; the environment variable
 *   ODMD_CORE_SVD=jacobi, read here, selects Jacobi only (diagnostics).
 *   workspace / workspace_bytes: NULL/0 to let the library allocate, else
 *          a device buffer of at least odmd_state_bytes(...) bytes, 256-byte
 *          aligned, owned by the caller and kept alive until odmd_destroy.
 *   Either way the handle also holds 64 bytes of pinned host memory, into
 *   which the device reports the rank after each update; the host sizes the
 *   next launches from it (work follows the live rank, not r_max).  Those
 *   words come from a per-device pool that lives until the process ends.
 *   The state is initialised by work queued on hip_stream (a memset and a
 *   one-thread kernel): creating a handle does not wait for the stream, and
 *   a device error of that work is reported by a later call.
 */
odmd_status odmd_create_ex(int64_t n, int32_t r_max, double tol, odmd_dtype basis,
                           odmd_dtype io, void* hip_stream, void* workspace,
                           size_t workspace_bytes, odmd_t* h);

/* Device bytes one handle needs (0 for invalid arguments). */
size_t odmd_state_bytes(int64_t n, int32_t r_max, odmd_dtype basis, odmd_dtype io);

/*
 * General pairs (Sec. 2.3 with U+ and U- built from pairs that need not
 * chain: several trajectories, or a hybrid run in which accepted
 * predictions replace full-order steps, so that x_k of a pair is not the
 * x_k1 of the pair before).  Arguments, memory and errors as for
 * odmd_create_ex.  The handle keeps B = Y W (n x r, Y the matrix of all
 * x_k1, W the right singular vectors) beside U, in the same stored-column
 * form (a second set of stored columns, appended with each x_k1 and
 * refolded when full), and A~ = U^T B S^-1.  Each update recomputes
 * U^T x_k with an extra sweep over the stored columns (the chained form
 * reuses the previous step's U^T x_k1), so it moves about twice the bytes
 * of a chained update; no chaining check is made.  odmd_update_batch
 * rejects such handles (ODMD_EINVAL); every other call works as for a
 * chained handle, the prediction anchored at the last x_k1.
 */
odmd_status odmd_create_general(int64_t n, int32_t r_max, double tol, odmd_dtype basis,
                                odmd_dtype io, void* hip_stream, void* workspace,
                                size_t workspace_bytes, odmd_t* h);

/* Device bytes of a general-pair handle (0 for invalid arguments). */
size_t odmd_state_bytes_general(int64_t n, int32_t r_max, odmd_dtype basis, odmd_dtype io);

/*
 * Launch shape of the streaming pass (the sweep over the n rows that does
 * the projections and CGS2 of Sec. 2.3 on the GPU): threads per workgroup
 * (256 or 512, the sizes the pass is compiled for) and one workgroup per
 * rows_per_block rows (a multiple of 16, at least 16, at most 2^24), at
 * most max_blocks workgroups (1..65536).  The partition of the rows sets
 * the order of the pass's sums, so a handle keeps its shape for life and
 * two handles fed the same pairs give bitwise equal results exactly when
 * their shapes give the same workgroup count and size (with the 512-thread
 * size, BF16 bases and FP32 bases of n >= 1,482,911, about 2^20.5, read
 * two rows per lane, also fixed per handle).  Results of any two shapes
 * agree to rounding.
 *
 * odmd_default_shape: the shape odmd_create_ex / odmd_create_general use
 * for n (512 x 256 rows, at most 256 workgroups, for n >= 131072; else
 * 256 x 512 rows, at most 512).  Host only.  ODMD_EINVAL for n < 1 or a
 * NULL output.
 */
odmd_status odmd_default_shape(int64_t n, int32_t* threads, int32_t* rows_per_block,
                               int32_t* max_blocks);

/*
 * As odmd_create_ex (general = 0) or odmd_create_general (general = 1),
 * with the pass's launch shape given explicitly (a tuned one, see
 * odmd_autotune).  ODMD_EINVAL for a shape outside the bounds above or a
 * general flag other than 0/1; memory and other errors as for
 * odmd_create_ex.
 */
odmd_status odmd_create_shaped(int64_t n, int32_t r_max, double tol, odmd_dtype basis,
                               odmd_dtype io, void* hip_stream, int32_t threads,
                               int32_t rows_per_block, int32_t max_blocks, int32_t general,
                               void* workspace, size_t workspace_bytes, odmd_t* h);

/* Device bytes of a handle with that shape (0 for invalid arguments). */
size_t odmd_state_bytes_shaped(int64_t n, int32_t r_max, odmd_dtype basis, odmd_dtype io,
                               int32_t threads, int32_t rows_per_block, int32_t max_blocks,
                               int32_t general);

/*
 * Autotuner of the pass's launch shape (not part of the method: it picks
 * how the sweep of Sec. 2.3's update is cut into workgroups).  It times
 * every candidate shape (threads 256 and 512; rows per workgroup 128 to
 * 2048; at most 256, 512 or 1024 workgroups; candidates that give the same
 * workgroup count and size are timed once) on chained handles of size n
 * and rank cap r_max fed seeded uniform random snapshots, so that the rank
 * saturates at r_max, the case that moves the most bytes:
 *   streams == 1: one handle, odmd_update calls one at a time; the figure
 *                 is the time per update (pass, core and the gap between);
 *   streams > 1 (at most 1024): that many handles of the same size
 *                 advanced by odmd_update_batch; the figure is the time
 *                 per batched step (a throughput objective).
 * Each candidate runs its warm-up (r_max + 24 updates) and then 48 timed
 * steps (three refold cycles at r = r_max) between HIP events on
 * hip_stream (NULL: the default stream); the shape with the least time
 * wins if it beats the default shape by more than 2 % (else the default
 * stays: a shape fixes the order of the sums, and smaller differences are
 * within the timing noise).  Outputs (host pointers): the
 * winning shape; *us_best its time and *us_default that of the default
 * shape (µs per update or per step).  Synchronous; allocates and frees its
 * own device memory (snapshots and handles), so it must not be called
 * while the stream is being captured.  ODMD_EINVAL for invalid sizes or
 * types or a NULL output, ODMD_ENOMEM when the handles or the
 * (r_max + 24) x n snapshots do not fit, ODMD_EDEVICE for runtime errors,
 * or the first error a timed handle reports.
 */
odmd_status odmd_autotune(int64_t n, int32_t r_max, odmd_dtype basis, odmd_dtype io,
                          int32_t streams, void* hip_stream, int32_t* threads,
                          int32_t* rows_per_block, int32_t* max_blocks, double* us_best,
                          double* us_default);

/*
 * Append one snapshot pair: x_k (a new column of U-) and x_k+1 (a new
 * column of U+); Sec. 2.3 grows each snapshot matrix by one column per
 * iteration, a rank-1 update.  x_k, x_k1: device, n elements of the io
 * type, contiguous; they must stay valid until the stream has run the
 * update.  The first call initialises the model from x_k (Sec. 2.1).
 * On a chained handle (odmd_create, odmd_create_ex) later pairs must
 * chain: x_k must equal, element for element, the x_k1 of the previous
 * accepted update; otherwise the update is skipped and ODMD_ESEQ is
 * latched.  The device checks two fingerprints, both summed in the same
 * fixed order by every pass of the handle: x.x, and a weighted sum with
 * weights in [1, 2) hashed from the row index (a sign flip or a
 * permutation of x changes it); a different x that matches both bit for
 * bit is not detected.  A general-pair handle (odmd_create_general) takes
 * any pair.
 * Asynchronous.  It may be captured into a HIP graph (stream capture on the
 * handle's stream): the graph then reads the same x_k, x_k1 buffers at
 * every replay, and from the capture on the handle sizes its passes for
 * the full stored-column capacity, as under a plan (results unchanged);
 * captured updates record no profiling events.
 */
odmd_status odmd_update(odmd_t h, const void* x_k, const void* x_k1);

/*
 * Append one pair to each of `count` handles: Sec. 2.3's rank-1 update
 * (as odmd_update) of every handle in one batched step.  The streaming
 * passes of all handles run as one launch per group of handles with the
 * same launch shape, storage type and live-column bucket (the groups'
 * launches on up to four side streams of default priority, joined to the
 * handles' stream), then one launch runs every handle's small-state update.
 * All handles must share one device and one HIP stream (that of hs[0]);
 * duplicates are not allowed.  hs, xs, ys: host arrays of length count;
 * xs[i], ys[i] are device pointers as in odmd_update.  Results are
 * identical, bit for bit, to calling odmd_update on each handle.
 * Asynchronous.  Its descriptor tables are staged through host memory, so
 * it returns ODMD_EINVAL while the stream is being captured: capture a
 * plan's launch instead (odmd_plan_create below).
 */
odmd_status odmd_update_batch(odmd_t* hs, const void* const* xs, const void* const* ys,
                              int32_t count);

/*
 * For callers that cannot allocate (tight serving loops, harnesses that
 * forbid hipMalloc): odmd_update_batch without any allocation.  Arguments,
 * results (bit for bit) and errors as odmd_update_batch, with count at most
 * ODMD_NOALLOC_MAX_STREAMS (ODMD_EINVAL above it).  The descriptor tables
 * of the launch live in a fixed device array of the library, one per GPU,
 * 208 KB, held until the process ends, instead of staging memory
 * the library allocates and grows; every pass launch goes to the handles'
 * stream (no side streams).  The tables are copied from a static host
 * buffer of the library, and the call waits for the handles' stream before
 * it returns (the work queued before it, not the update it queues), so
 * calls from several host threads are serialised.  Every call on one GPU
 * shares that GPU's array, which keeps the last call's tables: calls that
 * overlap on one GPU, from handles on different streams, race (the first
 * call's kernels may read the second call's tables).  Not capturable
 * (ODMD_EINVAL while the stream is being captured): capture a plan's
 * launch instead.  The first call on a device also looks up the array's
 * address on that device (no allocation).
 */
#define ODMD_NOALLOC_MAX_STREAMS 1024
odmd_status odmd_update_batch_noalloc(odmd_t* hs, const void* const* xs, const void* const* ys,
                                      int32_t count);

/*
 * Plans: one batched step (Sec. 2.3's rank-1 update of every handle, as
 * odmd_update_batch) fixed once, so that it can be launched again and
 * again with no host staging, host wait or allocation, and captured into
 * a HIP graph (hipStreamBeginCapture on the handles' stream, or a
 * framework's graph capture on that stream) and replayed.
 *
 * odmd_plan_create: hs, xs, ys, count as for odmd_update_batch (count >= 1,
 *   one stream and device, no duplicates, chained handles only); the
 *   pointers xs[i], ys[i] are fixed in the plan: the caller refills those
 *   device buffers between launches, keeping each pair chained (e.g. two
 *   plans over two buffers, used alternately: (A, B), then (B, A)).  The
 *   plan copies its descriptor tables to the device here (synchronous).
 *   A graph cannot follow the live stored-column count from the host, so
 *   each workgroup of a plan's passes reads its stream's count on the
 *   device and runs that count's live-column variant; from then on the
 *   handles size their own updates for the full capacity (the host no
 *   longer knows the count).  Results equal odmd_update_batch's bit for
 *   bit.  *plan is set to NULL on error; ODMD_EINVAL for invalid
 *   arguments, ODMD_ENOMEM if the tables or side streams cannot be made.
 * odmd_plan_launch: enqueue one step on the handles' stream (kernel
 *   launches, and event records and waits between that stream and the
 *   plan's own side streams, nothing else).  Asynchronous; errors latch in
 *   the handles as for odmd_update.
 * odmd_plan_destroy: wait for the stream, free the plan.  odmd_destroy of
 *   a handle that a live plan holds returns ODMD_EINVAL.
 */
typedef struct odmd_plan_s* odmd_plan_t;

odmd_status odmd_plan_create(odmd_t* hs, const void* const* xs, const void* const* ys,
                             int32_t count, odmd_plan_t* plan);
odmd_status odmd_plan_launch(odmd_plan_t plan);
odmd_status odmd_plan_destroy(odmd_plan_t plan);

/*
 * Eigenpairs of A~ (synchronising): the eigendecomposition A~ = V Lambda V^-1
 * of Sec. 2.3, whose columns of V give the projected DMD modes Phi = U V.
 * cap: capacity of the output arrays
 * (eigenvalue count; V arrays hold cap*cap doubles).  Outputs (host):
 *   *r        current rank;
 *   lam_re/im eigenvalues, |lambda| descending, then Im descending;
 *   v_re/v_im nullable; column j (r doubles, leading dimension r) is the
 *             eigenvector of lambda_j with unit 2-norm, scaled so that its
 *             largest-modulus entry is real and positive.  Without them the
 *             device computes the eigenvalues only (no Schur vectors or
 *             eigenvectors; the same eigenvalues bit for bit).
 * Returns ODMD_EEMPTY at rank 0, ODMD_EINVAL if cap < r.
 */
odmd_status odmd_eigs(odmd_t h, int32_t cap, int32_t* r, double* lam_re, double* lam_im,
                      double* v_re, double* v_im);

/*
 * Predicted states x_{a+1} .. x_{a+steps} where a is the time index of the
 * last x_k1 (Sec. 2.3, u(t) = Phi Lambda^(t/dt) Phi^+ u(0), anchored at the
 * last snapshot: Phi^+ u(0) = V^-1 U^T x_a).  At integer steps this is
 * U V Lambda^k V^-1 U^T x_a = U A~^k U^T x_a, which is how it is formed
 * (powers of A~, no eigendecomposition; the same states wherever A~ has a
 * full set of eigenvectors, and defined where it has not).  out: device,
 * steps x n, row k-1 holds state a+k, io type, row-major (row stride n).
 * steps >= 1.  Asynchronous; kernel launches only, so it may be captured
 * into a HIP graph.
 */
odmd_status odmd_predict(odmd_t h, int32_t steps, void* out);

/*
 * odmd_predict for several streams at once: the coefficients of every
 * stream's first chunk of states are formed in one launch (one workgroup
 * per stream), then each stream's states are written as by odmd_predict.  hs[i] distinct handles sharing one
 * device and HIP stream, steps[i] >= 1, outs[i] as odmd_predict's out (host
 * arrays of count entries, read during the call).  Asynchronous; results
 * equal those of odmd_predict bit for bit.  ODMD_EINVAL for a NULL entry,
 * steps < 1, a repeated handle or handles on different streams, and while
 * the stream is being captured (the handle table is staged through host
 * memory; odmd_predict itself may be captured).
 */
odmd_status odmd_predict_batch(odmd_t* hs, const int32_t* steps, void* const* outs, int32_t count);

/* Wait for the handle's stream; return and clear a latched error. */
odmd_status odmd_sync(odmd_t h);

/*
 * The error latched by the handle's finished device work, without waiting
 * and without any device call (a request loop that tracks completion with
 * its own events reads it per handle once that work is known to be done).
 * Every kernel that latches an error bit (an update skipped for a
 * non-finite or unchained pair, an iteration cap, a prediction of an empty
 * model) also writes the latched bits into a word of the handle's pinned
 * host memory; *status receives them as odmd_sync would return them (ODMD_OK
 * if none).  Work still in flight may not be reflected yet.  Does not clear
 * the error: odmd_sync (or odmd_eigs) does.  ODMD_EINVAL for NULL arguments.
 */
odmd_status odmd_peek_status(odmd_t h, odmd_status* status);

/* Free the handle and (unless caller-owned) its device memory, after
 * waiting for its stream; ODMD_EINVAL while a plan holds it. */
odmd_status odmd_destroy(odmd_t h);

/* Free the handle without waiting for its stream (a request loop that closes
 * many streams while others keep running; not a passage of the method).
 * A handle whose device memory the library allocated is destroyed as by
 * odmd_destroy (freeing device memory waits).  For a caller-owned
 * workspace the caller keeps the buffer until the work queued on the
 * handle's stream has finished: releasing it to an allocator that orders
 * reuse on that same stream (torch's caching allocator, for a handle made
 * on torch's current stream) is enough.  The handle's pinned host word
 * goes back to a pool once that work has finished (an event on the stream).
 * Errors of the queued work are not reported here.  ODMD_EINVAL for NULL or
 * while a plan holds the handle. */
odmd_status odmd_release(odmd_t h);

const char* odmd_status_str(odmd_status s);

/* ---- introspection (synchronising; for tests, diagnostics, benchmarks) ---- */

typedef struct {
  int32_t r;          /* current rank                                   */
  int32_t r_max;
  int64_t n;
  int64_t m;          /* accepted pairs                                 */
  double tol_eff;     /* tolerance in use (after the BF16 floor)        */
  double last_rho;    /* residual norm of the last accepted update      */
  int32_t last_sweeps;/* Jacobi sweeps of the last small SVD            */
  int32_t nblocks;    /* workgroups of the streaming pass               */
  int32_t threads;    /* threads per workgroup of the streaming pass    */
  int32_t stored;     /* stored basis columns in use (U = S[:, :stored] Q) */
  int32_t capacity;   /* stored-column capacity: min(72, r_max + 16 rounded
                         up to 8); FP64/FP32 bases refold at r + 16 stored
                         columns already, BF16 bases at the capacity      */
} odmd_info;

odmd_status odmd_get_info(odmd_t h, odmd_info* info);

/*
 * Copy the small state to host arrays (any may be NULL): sigma (r),
 * A~ (r x r, column-major, leading dimension r), p_y = U^T x_a (r),
 * C (r x r, column-major) and w (r), the shifted product of the right
 * singular vectors and their last row.
 */
odmd_status odmd_get_state(odmd_t h, int32_t cap, double* sigma, double* atilde, double* p_y,
                           double* C, double* w);

/* The current basis U as FP64, device out: n x r column-major with
 * leading dimension n (needs n * r_max doubles).  Asynchronous. */
odmd_status odmd_get_basis(odmd_t h, double* out);

/*
 * Kernel timing.  odmd_profile(h, capacity) with capacity > 0 creates HIP
 * events for at least `capacity` updates (up front, so that timing adds no
 * allocation later) and makes every later update launch its streaming pass
 * and its small-SVD kernel with a start and an end event each, which take
 * the kernel's own begin and end timestamps; capacity 0 stops recording.
 * odmd_profile_read (synchronising) returns the summed pass and core
 * durations in milliseconds and the number of timed updates, then resets.
 */
odmd_status odmd_profile(odmd_t h, int32_t capacity);
odmd_status odmd_profile_read(odmd_t h, double* pass_ms, double* core_ms, int64_t* count);

/* Per-update samples instead of sums (synchronising): pass_ms[k], core_ms[k]
 * and update_ms[k] (pass start to core end, including the launch gap
 * between the two; update_ms may be NULL) for the first
 * min(cap, timed updates) updates (host arrays of length cap); *count
 * receives the number of timed updates.  Resets like odmd_profile_read. */
odmd_status odmd_profile_samples(odmd_t h, int64_t cap, double* pass_ms, double* core_ms,
                                 double* update_ms, int64_t* count);

/* Latency-only timing (a measurement aid, not a passage of the method):
 * while on != 0, a timed update records only its pass's start and its
 * small-SVD kernel's end, so that no event sits between the two kernels (an
 * event there delays the second launch by several microseconds on MI355X).
 * Such an update's pass_ms and core_ms samples read as NaN and
 * odmd_profile_read leaves it out of its sums and count; update_ms is its
 * latency.  EINVAL for a NULL handle. */
odmd_status odmd_profile_latency(odmd_t h, int32_t on);

#ifdef __cplusplus
}
#endif
#endif /* ODMD_H */
