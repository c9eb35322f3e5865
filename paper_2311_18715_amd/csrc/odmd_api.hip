// Host runtime behind the C ABI declared in include/odmd.h.
//
// Every entry point validates its arguments on the host before touching the
// device, queues its kernels on the handle's HIP stream, and reports HIP
// runtime failures as ODMD_EDEVICE.  Errors that only the GPU can see are
// latched in DevState::status and surface at the next synchronising call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <cmath>
#include <cstddef>
#include <cstdlib>
#include <cstring>
#include <new>
#include <unordered_set>
#include <tuple>
#include <vector>

#include "odmd.h"
#include "odmd_internal.h"
#include "pass.h"

using namespace odmd;

constexpr size_t EV_PER_UPDATE = 4;   // timing events of one profiled update

struct odmd_s {
  int64_t n = 0;
  int r_max = 0, ct = 0;      // rank cap, stored-column capacity of the tiles
  double tol = 0.0, tol_eff = 0.0;
  odmd_dtype basis = ODMD_F64, io = ODMD_F64;
  hipStream_t stream = nullptr;
  int device = 0;
  char* mem = nullptr;
  size_t bytes = 0;
  bool own = false;
  DevState* st = nullptr;
  double* partials = nullptr;
  void* Us = nullptr;
  // general pairs: B = Y W held as T R (stored y columns T, R in tst->Q),
  // records of the projection sweep and of the T sweep
  bool general = false;
  DevState* tst = nullptr;
  void* Ts = nullptr;
  double* pproj = nullptr;
  double* pt = nullptr;
  void* eout = nullptr;         // the residual e as a contiguous vector (io type)
  int nblk = 0;
  int threads = 0;              // workgroup size of the stream's pass launch shape
  int rows2 = 0;                // the pass's wide-row variant (PassArgs::rows2)
  int64_t units = 0;
  bool prof = false;
  bool jacobi_only = false;     // ODMD_CORE_SVD=jacobi at create time
  std::vector<hipEvent_t> ev;   // per update: pass start, pass end, core start, core end
  size_t ev_used = 0;
  bool prof_lat = false;        // timed updates record the pass start and the core end only
  std::vector<unsigned char> ev_lat;   // per timed update: recorded with prof_lat
  // Feedback: the core writes (seq << 8) | m (stored columns in use) into
  // this pinned host word after every update; seq counts the updates issued
  // on the handle.
  unsigned* fb_host = nullptr;
  unsigned* fb_dev = nullptr;
  // BF16 basis: records of the Gram kernel that follows each pass (the Gram
  // matrix of the columns a refold rewrote), gnwg of them
  double* grec = nullptr;
  int gnwg = 0;
  unsigned seq = 0;
  // Set once a plan holds the handle: plan launches (possibly replayed from
  // a graph) advance the state without the host's count, so every later
  // pass is sized for the full stored-column capacity.
  bool full_bucket = false;
  int plans = 0;                // live plans that hold the handle
};

namespace {

struct Layout {
  size_t st = 0, partials = 0, Us = 0, total = 0;
  size_t gram = 0;   // BF16 basis: Gram records
  int gnwg = 0;
  size_t tst = 0, pproj = 0, pt = 0, Ts = 0, eout = 0;   // general pairs only
  int64_t ntiles = 0, units = 0;
  int nblk = 0, ct = 0, threads = 0;
};

int elem_bytes(odmd_dtype t) { return t == ODMD_F64 ? 8 : (t == ODMD_F32 ? 4 : 2); }

// F64 and F32 bases take snapshots of their own type; a BF16 basis takes
// F32 snapshots.
bool valid_types(odmd_dtype basis, odmd_dtype io) {
  if (basis == ODMD_BF16) return io == ODMD_F32;
  if (basis != ODMD_F64 && basis != ODMD_F32) return false;
  return io == basis;
}

bool valid_args(int64_t n, int32_t r_max, double tol, odmd_dtype basis, odmd_dtype io) {
  if (n < 1 || n > (int64_t(1) << 40)) return false;
  if (r_max < 1 || r_max > RMAX || (int64_t)r_max > n) return false;
  if (!std::isfinite(tol) || tol < 0.0 || tol >= 1.0) return false;
  return valid_types(basis, io);
}

int col_bucket(int cols) { return (cols + 7) / 8 * 8; }

// Two rows per lane in the 512-thread pass: always for BF16 storage (half
// lines instead of quarter lines per load), for FP32 storage only from
// about 2^20.5 rows on (1,482,911 = the first n whose nearest power of two
// in log scale is 2^21, so that a tuned-shape bucket never mixes the two
// variants).  A single HBM-bound stream gains (whole lines: the n = 6M
// FP32 update 521 -> 481 us), while the higher register count costs
// batches: at n = 2^21, r_max 16, a 16-stream batch step went from 874 to
// 941 us with the 512-thread shape (the tuned table picks each bucket's
// shape with the variant in effect); below this size, where the batched
// mixes live, one row per lane stays.
constexpr int64_t F32_WIDE_ROWS_MIN_N = 1482911;
int wide_rows(odmd_dtype basis, int threads, int64_t n) {
  if (threads != PASS_WIDE.threads) return 0;
  return basis == ODMD_BF16 || (basis == ODMD_F32 && n >= F32_WIDE_ROWS_MIN_N);
}

// Stored basis: 64-row tiles, column-major inside a tile, fold_capacity(r_max)
// columns per tile.
// The pass's workgroups: one per rows_per_block rows, at most max_blocks;
// each gets at least one 16-row unit (rows_per_block >= 16).
Layout make_layout(int64_t n, int32_t r_max, odmd_dtype basis, bool general, const PassShape& sh) {
  Layout L;
  L.ct = fold_capacity(r_max);
  L.ntiles = (n + 63) / 64;
  L.threads = sh.threads;
  L.units = (n + sh.rows_per_block - 1) / sh.rows_per_block;
  L.nblk = (int)std::min<int64_t>(L.units, sh.max_blocks);
  size_t off = 0;
  L.st = off;
  off += round_up(sizeof(DevState), 256);
  L.partials = off;
  off += round_up((int64_t)L.nblk * PW * sizeof(double), 256);
  L.Us = off;
  off += round_up(L.ntiles * L.ct * 64 * elem_bytes(basis), 256);
  if (basis == ODMD_BF16) {
    L.gnwg = gram_workgroups(n);
    L.gram = off;
    off += round_up((int64_t)L.gnwg * GRAM_REC * sizeof(double), 256);
  }
  if (general) {
    L.tst = off;
    off += round_up(sizeof(DevState), 256);
    L.pproj = off;
    off += round_up((int64_t)L.nblk * PW * sizeof(double), 256);
    L.pt = off;
    off += round_up((int64_t)L.nblk * PW * sizeof(double), 256);
    L.Ts = off;
    off += round_up(L.ntiles * L.ct * 64 * elem_bytes(basis), 256);
    L.eout = off;
    off += round_up(n * 8, 256);
  }
  L.total = off;
  return L;
}

odmd_status map_status(int bits) {
  if (bits & ST_NONFINITE) return ODMD_ENONFINITE;
  if (bits & ST_SEQ) return ODMD_ESEQ;
  if (bits & ST_NOCONV) return ODMD_ENOCONV;
  if (bits & ST_EMPTY) return ODMD_EEMPTY;
  return ODMD_OK;
}

#define HIP_OK(expr)                        \
  do {                                      \
    if ((expr) != hipSuccess) {             \
      (void)hipGetLastError();              \
      return ODMD_EDEVICE;                  \
    }                                       \
  } while (0)

// Wait for the stream, then fetch and clear the latched device status.
odmd_status sync_and_status(odmd_t h) {
  HIP_OK(hipStreamSynchronize(h->stream));
  int bits = 0;
  HIP_OK(hipMemcpy(&bits, &h->st->status, sizeof(int), hipMemcpyDeviceToHost));
  if (bits) {
    const int zero = 0;
    HIP_OK(hipMemcpy(&h->st->status, &zero, sizeof(int), hipMemcpyHostToDevice));
    __atomic_store_n(h->fb_host + 1, 0u, __ATOMIC_RELEASE);   // the host-visible copy too
  }
  return map_status(bits);
}

template <typename T>
odmd_status copy_field(odmd_t h, T* dst, const T* src_dev, size_t count) {
  HIP_OK(hipMemcpyAsync(dst, src_dev, count * sizeof(T), hipMemcpyDeviceToHost, h->stream));
  return ODMD_OK;
}

// Refold slack of the core (CoreArgs::fold_slack): FP64 and FP32 bases
// refold once FOLD_SLACK columns are pending; a BF16 basis only at the
// capacity, since every refold rounds the basis to BF16 again.
int fold_slack(odmd_t h) { return h->basis == ODMD_BF16 ? 0 : FOLD_SLACK; }

// Live-column bucket for the next pass: an upper bound on the stored
// columns in use after the last issued update.  They grow by at most one per
// update, so the last count the device reported plus the number of updates
// issued since bounds them.  The bucket is a multiple of 8 and never exceeds
// the tile capacity.
int live_bucket(odmd_t h) {
  if (h->full_bucket) return h->ct;
  const unsigned v = __atomic_load_n(h->fb_host, __ATOMIC_ACQUIRE);
  const unsigned lag = (h->seq - (v >> 8)) & 0xFFFFFFu;
  const int64_t bound = std::min<int64_t>(h->ct, (int64_t)(v & 0xFFu) + lag);
  return std::max(8, col_bucket((int)bound));
}

// True while the stream is being captured into a graph.
bool capturing(hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return cs != hipStreamCaptureStatusNone;
}

GramArgs gram_args(odmd_t h) {
  GramArgs g{};
  g.st = h->st;
  g.Us = h->Us;
  g.rec = h->grec;
  g.n = h->n;
  g.ct = h->ct;
  g.nwg = h->gnwg;
  g.blk0 = 0;
  return g;
}

// The Gram kernels of the BF16 handles among hs[0..count), in index order,
// into out (count entries at most); returns their number, *nblocks the
// workgroups of one batched launch.
int fill_gram(odmd_t* hs, int32_t count, GramArgs* out, int* nblocks) {
  int k = 0, blk = 0;
  for (int32_t i = 0; i < count; ++i) {
    if (!hs[i]->grec) continue;
    out[k] = gram_args(hs[i]);
    out[k].blk0 = blk;
    blk += hs[i]->gnwg;
    ++k;
  }
  *nblocks = blk;
  return k;
}

odmd_status launch_update(odmd_t h, const void* x, const void* y) {
  // a captured update is replayed without the host's count of stored
  // columns: from here on the passes are sized for the full capacity (and
  // no timing events are recorded into the graph)
  const bool cap = capturing(h->stream);
  if (cap) h->full_bucket = true;
  hipEvent_t* ev = nullptr;
  if (h->prof && !cap) {
    if (h->ev_used + EV_PER_UPDATE > h->ev.size()) {
      for (int k = 0; k < EV_PER_UPDATE; ++k) {
        hipEvent_t e;
        HIP_OK(hipEventCreate(&e));
        h->ev.push_back(e);
      }
    }
    ev = &h->ev[h->ev_used];
    h->ev_used += EV_PER_UPDATE;
    h->ev_lat.push_back(h->prof_lat ? 1 : 0);
  }
  const bool lat = ev && h->prof_lat;   // no events between the two kernels
  PassArgs p{};
  p.Us = h->Us;
  p.x = x;
  p.y = y;
  p.partials = h->partials;
  p.st = h->st;
  p.n = h->n;
  p.units = h->units;
  p.nblk = h->nblk;
  p.ct = h->ct;
  p.threads = h->threads;
  p.rows2 = h->rows2;
  const int kb = live_bucket(h);
  if (h->general) {
    // U^T x from a projection sweep, then the coefficients of the streaming
    // pass (which also writes e contiguously for the T sweep below)
    PassArgs pp = p;
    pp.partials = h->pproj;
    HIP_OK(launch_proj(pp, (int)h->basis, kb, h->stream));
    CoefArgs ca{};
    ca.st = h->st;
    ca.pproj = h->pproj;
    ca.nblk = h->nblk;
    ca.rb = kb;
    HIP_OK(launch_coef(ca, h->stream));
    p.eout = h->eout;
  }
  HIP_OK(launch_pass(p, (int)h->basis, kb, h->stream, ev ? ev[0] : nullptr, ev && !lat ? ev[1] : nullptr));
  if (h->general) {
    // the T sweep: appends y to T (refolding T when it is full) with zero
    // coefficients; its records carry T^T e
    PassArgs pt = p;
    pt.Us = h->Ts;
    pt.x = y;
    pt.y = h->eout;
    pt.partials = h->pt;
    pt.st = h->tst;
    pt.eout = nullptr;
    HIP_OK(launch_pass(pt, (int)h->basis, h->ct, h->stream));
  }
  if (h->grec) HIP_OK(launch_gram(gram_args(h), h->stream));
  h->seq = (h->seq + 1) & 0xFFFFFFu;
  CoreArgs c{};
  c.st = h->st;
  c.partials = h->partials;
  c.nblk = h->nblk;
  c.grec = h->grec;
  c.gnwg = h->gnwg;
  c.r_max = h->r_max;
  c.jacobi_only = h->jacobi_only;
  c.rb = kb;
  c.ct = h->ct;
  c.fold_slack = fold_slack(h);
  c.fb = h->fb_dev;
  c.seq = h->seq;
  c.tst = h->general ? h->tst : nullptr;
  c.pt = h->general ? h->pt : nullptr;
  c.rbt = h->ct;
  HIP_OK(launch_core(c, h->stream, ev && !lat ? ev[2] : nullptr, ev ? ev[3] : nullptr));
  return ODMD_OK;
}

// Descriptor tables of batched launches: a small ring of pinned host / device
// buffer pairs per device; a slot is reused only after the kernels that read
// its table have run, so the host queues at most NSLOT batched calls ahead
// of the device (32 slots took the 256-stream batched loop from 149.5k to
// 138.4k stream-updates/s).
struct BatchSlot {
  void* host = nullptr;
  void* dev = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;
  bool used = false;
};
constexpr int NSIDE = 4;   // side streams for the pass launches of one batch
constexpr int NSLOT = 4;   // staging slots per device
struct BatchRing {
  std::mutex mu;
  BatchSlot slot[NSLOT];
  int next = 0;
  // The pass launches of a batch's groups are independent: they go to side
  // streams (default priority) so that one launch's tail overlaps the next
  // launch; the core launch on the caller's stream waits for all of them.
  hipStream_t side[NSIDE] = {};
  hipEvent_t fork = nullptr, join[NSIDE] = {};
};
std::mutex g_ring_mu;
std::map<int, std::unique_ptr<BatchRing>> g_rings;

BatchRing* ring_for(int device) {
  std::lock_guard<std::mutex> lk(g_ring_mu);
  auto& p = g_rings[device];
  if (!p) p.reset(new BatchRing());
  return p.get();
}

// Next staging slot of the device's ring, grown to at least `bytes`; the
// ring stays locked (lk) until the caller has recorded the slot's event.
odmd_status acquire_slot(int device, size_t bytes, std::unique_lock<std::mutex>& lk, BatchSlot*& out,
                         BatchRing** ring_out = nullptr) {
  BatchRing* ring = ring_for(device);
  lk = std::unique_lock<std::mutex>(ring->mu);
  if (ring_out) {
    if (!ring->fork) {
      HIP_OK(hipEventCreateWithFlags(&ring->fork, hipEventDisableTiming));
      for (int i = 0; i < NSIDE; ++i) {
        HIP_OK(hipStreamCreateWithFlags(&ring->side[i], hipStreamNonBlocking));
        HIP_OK(hipEventCreateWithFlags(&ring->join[i], hipEventDisableTiming));
      }
    }
    *ring_out = ring;
  }
  BatchSlot& sl = ring->slot[ring->next];
  ring->next = (ring->next + 1) % NSLOT;
  if (sl.used) HIP_OK(hipEventSynchronize(sl.done));
  if (sl.cap < bytes) {
    if (sl.host) (void)hipHostFree(sl.host);
    if (sl.dev) (void)hipFree(sl.dev);
    sl.host = sl.dev = nullptr;
    sl.cap = 0;
    if (hipHostMalloc(&sl.host, bytes, hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&sl.dev, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return ODMD_ENOMEM;
    }
    sl.cap = bytes;
  }
  if (!sl.done) HIP_OK(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
  out = &sl;
  return ODMD_OK;
}

// Launch plan of a batched update.  Streams are grouped by launch shape,
// wide-row variant and storage type (one pass kernel each), and inside such
// a group by live-column bucket; a bucket group too small to fill the chip
// (fewer than BATCH_FILL workgroups) is merged into the next larger bucket
// of its group, whose pass reads more columns than it needs (the extra
// k-steps meet zero coefficients: results do not change by a bit), so that
// the batch makes fewer, fuller launches.  kb[i] is raised to the bucket
// stream i runs with (its small-state kernel reads records of that length).
// order receives the streams in launch order (per launch the most rows per
// workgroup first: workgroups start in index order, so the short ones fill
// in behind the long ones), out the launches; returns their count.  No
// allocation: order and out are caller arrays of count entries.
constexpr int BATCH_FILL = 512;
struct BatchLaunch { int first, nd, nblocks, threads, rows2, basis, rb; };
int plan_batch(odmd_t* hs, int* kb, int32_t count, int* order, BatchLaunch* out) {
  auto key = [&](int i) { return std::make_tuple(hs[i]->threads, hs[i]->rows2, (int)hs[i]->basis); };
  for (int32_t i = 0; i < count; ++i) order[i] = i;
  std::sort(order, order + count, [&](int a, int b) {
    if (key(a) != key(b)) return key(a) < key(b);
    if (kb[a] != kb[b]) return kb[a] < kb[b];
    return a < b;
  });
  int nl = 0;
  for (int a = 0; a < count;) {
    // [a, b): streams of one kernel group merged up to one bucket
    int b = a, nblk = 0;
    while (b < count && key(order[b]) == key(order[a])) {
      const int bucket = kb[order[b]];
      while (b < count && key(order[b]) == key(order[a]) && kb[order[b]] == bucket)
        nblk += hs[order[b++]]->nblk;
      if (nblk >= BATCH_FILL) break;
    }
    const int rb = kb[order[b - 1]];
    std::sort(order + a, order + b, [&](int x, int y) {
      const int64_t lx = hs[x]->n * hs[y]->nblk, ly = hs[y]->n * hs[x]->nblk;
      if (lx != ly) return lx > ly;
      return x < y;
    });
    out[nl++] = BatchLaunch{a, b - a, nblk, hs[order[a]]->threads, hs[order[a]]->rows2,
                            (int)hs[order[a]]->basis, rb};
    for (int k = a; k < b; ++k) kb[order[k]] = rb;
    a = b;
  }
  return nl;
}

odmd_status launch_batch(odmd_t* hs, const void* const* xs, const void* const* ys, int32_t count) {
  hipStream_t stream = hs[0]->stream;
  // one pass launch per group of plan_batch
  std::vector<int> kb(count);
  std::vector<int> order(count);
  std::vector<BatchLaunch> launches(count);
  for (int32_t i = 0; i < count; ++i) kb[i] = live_bucket(hs[i]);
  launches.resize(plan_batch(hs, kb.data(), count, order.data(), launches.data()));
  const size_t pass_bytes = round_up((int64_t)count * sizeof(PassDesc), 256);
  const size_t core_bytes = round_up((int64_t)count * sizeof(CoreArgs), 256);
  const size_t bytes = pass_bytes + core_bytes + (size_t)count * sizeof(GramArgs);
  std::unique_lock<std::mutex> lk;
  BatchSlot* slp = nullptr;
  BatchRing* ring = nullptr;
  {
    const odmd_status s = acquire_slot(hs[0]->device, bytes, lk, slp, &ring);
    if (s != ODMD_OK) return s;
  }
  BatchSlot& sl = *slp;
  PassDesc* pd = static_cast<PassDesc*>(sl.host);
  CoreArgs* cd = reinterpret_cast<CoreArgs*>(static_cast<char*>(sl.host) + pass_bytes);
  GramArgs* gd = reinterpret_cast<GramArgs*>(static_cast<char*>(sl.host) + pass_bytes + core_bytes);
  int gblocks = 0;
  const int ngram = fill_gram(hs, count, gd, &gblocks);
  for (const BatchLaunch& L : launches) {
    int blk0 = 0;
    for (int k = L.first; k < L.first + L.nd; ++k) {
      const int i = order[k];
      odmd_t h = hs[i];
      PassDesc& d = pd[k];
      d = PassDesc{};
      d.Us = h->Us;
      d.x = xs[i];
      d.y = ys[i];
      d.partials = h->partials;
      d.st = h->st;
      d.n = h->n;
      d.nblk = h->nblk;
      d.ct = h->ct;
      d.blk0 = blk0;
      blk0 += h->nblk;
    }
  }
  for (int32_t i = 0; i < count; ++i) {
    odmd_t h = hs[i];
    CoreArgs& c = cd[i];
    c = CoreArgs{};   // every field set below or zero (tst: chained handles only here)
    c.st = h->st;
    c.partials = h->partials;
    c.nblk = h->nblk;
    c.r_max = h->r_max;
    c.jacobi_only = h->jacobi_only;
    c.rb = kb[i];
    c.ct = h->ct;
    c.fold_slack = fold_slack(h);
    c.grec = h->grec;
    c.gnwg = h->gnwg;
    h->seq = (h->seq + 1) & 0xFFFFFFu;
    c.fb = h->fb_dev;
    c.seq = h->seq;
  }
  HIP_OK(hipMemcpyAsync(sl.dev, sl.host, bytes, hipMemcpyHostToDevice, stream));
  const PassDesc* dpd = static_cast<const PassDesc*>(sl.dev);
  if (launches.size() == 1) {
    const BatchLaunch& L = launches[0];
    HIP_OK(launch_pass_batch(dpd + L.first, L.nd, L.nblocks, L.threads, L.rows2, L.basis, L.rb, stream));
  } else {
    const int nside = std::min<int>(NSIDE, (int)launches.size());
    HIP_OK(hipEventRecord(ring->fork, stream));
    for (int i = 0; i < nside; ++i) HIP_OK(hipStreamWaitEvent(ring->side[i], ring->fork, 0));
    for (size_t i = 0; i < launches.size(); ++i) {
      const BatchLaunch& L = launches[i];
      HIP_OK(launch_pass_batch(dpd + L.first, L.nd, L.nblocks, L.threads, L.rows2, L.basis, L.rb,
                               ring->side[i % nside]));
    }
    for (int i = 0; i < nside; ++i) {
      HIP_OK(hipEventRecord(ring->join[i], ring->side[i]));
      HIP_OK(hipStreamWaitEvent(stream, ring->join[i], 0));
    }
  }
  if (ngram > 0)
    HIP_OK(launch_gram_batch(reinterpret_cast<const GramArgs*>(static_cast<char*>(sl.dev) + pass_bytes +
                                                               core_bytes),
                             ngram, gblocks, stream));
  HIP_OK(launch_core_batch(reinterpret_cast<const CoreArgs*>(static_cast<char*>(sl.dev) + pass_bytes),
                           count, stream));
  // the slot (host staging and device table) is free again once the
  // kernels that read the table have run
  HIP_OK(hipEventRecord(sl.done, stream));
  sl.used = true;
  return ODMD_OK;
}

// ---- the batched update without allocation (odmd_update_batch_noalloc) ----
//
// Its descriptor tables live in `scratch`, one file-scope device array per
// GPU (held until the process ends), instead of a ring slot the library
// grows with hipMalloc; every pass launch goes to the caller's stream (no
// side streams); the host staging is a static buffer of this library.  The
// device address of each GPU's copy of `scratch` is taken once per device
// (hipGetSymbolAddress, that device current) and used wherever host code
// names the array's memory.
constexpr int NOALLOC_MAX = ODMD_NOALLOC_MAX_STREAMS;
constexpr size_t NOALLOC_PASS_BYTES = (NOALLOC_MAX * sizeof(PassDesc) + 255) / 256 * 256;
constexpr size_t NOALLOC_CORE_BYTES = (NOALLOC_MAX * sizeof(CoreArgs) + 255) / 256 * 256;
constexpr size_t NOALLOC_BYTES = NOALLOC_PASS_BYTES + NOALLOC_CORE_BYTES + NOALLOC_MAX * sizeof(GramArgs);
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int NOALLOC_DEVICES = 64;
std::mutex g_noalloc_mu;                      // guards the two tables below
void* g_scratch_ptr[NOALLOC_DEVICES] = {};    // per device: its copy of scratch
alignas(256) unsigned char g_noalloc_host[NOALLOC_BYTES];   // host staging (pageable)

// Caller holds g_noalloc_mu; the device is current.
odmd_status scratch_for(int device, unsigned char** out) {
  if (device < 0 || device >= NOALLOC_DEVICES) return ODMD_EDEVICE;
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    HIP_OK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return ODMD_EDEVICE;
    g_scratch_ptr[device] = ptr;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[device]);
  return ODMD_OK;
}

odmd_status launch_batch_noalloc(odmd_t* hs, const void* const* xs, const void* const* ys,
                                 int32_t count) {
  hipStream_t stream = hs[0]->stream;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  unsigned char* dev = nullptr;
  {
    const odmd_status s = scratch_for(hs[0]->device, &dev);
    if (s != ODMD_OK) return s;
  }
  // the launch plan of odmd_update_batch (plan_batch), in stack arrays
  int kb[NOALLOC_MAX], order[NOALLOC_MAX];
  BatchLaunch launches[NOALLOC_MAX];
  for (int32_t i = 0; i < count; ++i) kb[i] = live_bucket(hs[i]);
  const int nl = plan_batch(hs, kb, count, order, launches);
  PassDesc* pd = reinterpret_cast<PassDesc*>(g_noalloc_host);
  CoreArgs* cd = reinterpret_cast<CoreArgs*>(g_noalloc_host + NOALLOC_PASS_BYTES);
  GramArgs* gd = reinterpret_cast<GramArgs*>(g_noalloc_host + NOALLOC_PASS_BYTES + NOALLOC_CORE_BYTES);
  int gblocks = 0;
  const int ngram = fill_gram(hs, count, gd, &gblocks);
  for (int l = 0; l < nl; ++l) {
    const BatchLaunch& L = launches[l];
    int blk0 = 0;
    for (int k = L.first; k < L.first + L.nd; ++k) {
      const int i = order[k];
      odmd_t h = hs[i];
      PassDesc& d = pd[k];
      d = PassDesc{};
      d.Us = h->Us;
      d.x = xs[i];
      d.y = ys[i];
      d.partials = h->partials;
      d.st = h->st;
      d.n = h->n;
      d.nblk = h->nblk;
      d.ct = h->ct;
      d.blk0 = blk0;
      blk0 += h->nblk;
    }
  }
  for (int32_t i = 0; i < count; ++i) {
    odmd_t h = hs[i];
    CoreArgs& c = cd[i];
    c = CoreArgs{};
    c.st = h->st;
    c.partials = h->partials;
    c.nblk = h->nblk;
    c.r_max = h->r_max;
    c.jacobi_only = h->jacobi_only;
    c.rb = kb[i];
    c.ct = h->ct;
    c.fold_slack = fold_slack(h);
    c.grec = h->grec;
    c.gnwg = h->gnwg;
    h->seq = (h->seq + 1) & 0xFFFFFFu;
    c.fb = h->fb_dev;
    c.seq = h->seq;
  }
  // Copy the used parts of the tables (pageable source: the copy completes
  // before the call returns, after the work queued on the stream before it,
  // which includes the kernels of an earlier call that read the tables);
  // the wait makes sure of that whatever the runtime does, so the static
  // staging buffer is free when the lock is released.
  const size_t pbytes = (size_t)count * sizeof(PassDesc), cbytes = (size_t)count * sizeof(CoreArgs);
  HIP_OK(hipMemcpyAsync(dev, g_noalloc_host, pbytes, hipMemcpyHostToDevice, stream));
  HIP_OK(hipMemcpyAsync(dev + NOALLOC_PASS_BYTES, g_noalloc_host + NOALLOC_PASS_BYTES, cbytes,
                        hipMemcpyHostToDevice, stream));
  if (ngram > 0)
    HIP_OK(hipMemcpyAsync(dev + NOALLOC_PASS_BYTES + NOALLOC_CORE_BYTES,
                          g_noalloc_host + NOALLOC_PASS_BYTES + NOALLOC_CORE_BYTES,
                          (size_t)ngram * sizeof(GramArgs), hipMemcpyHostToDevice, stream));
  HIP_OK(hipStreamSynchronize(stream));
  const PassDesc* dpd = reinterpret_cast<const PassDesc*>(dev);
  for (int l = 0; l < nl; ++l) {
    const BatchLaunch& L = launches[l];
    HIP_OK(launch_pass_batch(dpd + L.first, L.nd, L.nblocks, L.threads, L.rows2, L.basis, L.rb, stream));
  }
  if (ngram > 0)
    HIP_OK(launch_gram_batch(reinterpret_cast<const GramArgs*>(dev + NOALLOC_PASS_BYTES + NOALLOC_CORE_BYTES),
                             ngram, gblocks, stream));
  HIP_OK(launch_core_batch(reinterpret_cast<const CoreArgs*>(dev + NOALLOC_PASS_BYTES), count, stream));
  return ODMD_OK;
}

odmd_status launch_combine_cols(odmd_t h, void* out, int64_t ldo, int K, bool out_f32) {
  CombineArgs c{};
  c.st = h->st;
  c.Us = h->Us;
  c.out = out;
  c.n = h->n;
  c.ct = h->ct;
  c.ldo = ldo;
  c.K = K;
  // the live-column bucket (an upper bound on the stored columns in use):
  // fewer k-steps, and less LDS per workgroup for the staged coefficients
  HIP_OK(launch_combine(c, (int)h->basis, out_f32, live_bucket(h), h->stream));
  return ODMD_OK;
}

// Coefficients and read-out of predicted states a+1 .. a+steps, COEF_CHUNK
// states per read-out launch; their coefficients in launches of
// coef_chunk(r_max) states, each starting where the last one ended
// (first_done: the first of them is already queued, by a batched launch).
odmd_status launch_rollout(odmd_t h, int32_t steps, void* out, bool first_done = false) {
  const int es = elem_bytes(h->io);
  const int ch = coef_chunk(h->r_max);
  for (int k0 = 0; k0 < steps; k0 += COEF_CHUNK) {
    const int K = std::min(COEF_CHUNK, steps - k0);
    for (int j = 0; j < K; j += ch)
      if (k0 + j > 0 || !first_done) HIP_OK(launch_power_coef(h->st, k0 + j, std::min(ch, K - j), j, h->stream));
    char* o = static_cast<char*>(out) + (int64_t)k0 * h->n * es;
    const odmd_status s = launch_combine_cols(h, o, h->n, K, h->io == ODMD_F32);
    if (s != ODMD_OK) return s;
  }
  return ODMD_OK;
}

// ---- pinned feedback words: a per-device pool ----
// Each handle holds one 64-byte slot of mapped, coherent pinned host memory
// (the rank feedback and the status mirror).  Allocating and freeing pinned
// memory synchronises the device, so slots come from chunks that live until
// the process ends.  A slot given back while the handle's work may still
// write it waits behind an event recorded on the handle's stream.
struct FbPool {
  std::mutex mu;
  std::vector<std::pair<unsigned*, unsigned*>> free;                 // (host, device)
  std::vector<std::tuple<hipEvent_t, unsigned*, unsigned*>> waiting;
};
constexpr int FB_SLOT_WORDS = 16;     // 64 bytes
constexpr int FB_CHUNK_SLOTS = 1024;

FbPool& fb_pool(int device) {
  static std::mutex mu;
  static std::map<int, std::unique_ptr<FbPool>> pools;
  std::lock_guard<std::mutex> lk(mu);
  std::unique_ptr<FbPool>& p = pools[device];
  if (!p) p.reset(new FbPool);
  return *p;
}

// a zeroed slot of the current device, or false
bool fb_acquire(int device, unsigned** host, unsigned** dev) {
  FbPool& P = fb_pool(device);
  std::lock_guard<std::mutex> lk(P.mu);
  for (size_t i = 0; i < P.waiting.size();) {
    hipEvent_t e = std::get<0>(P.waiting[i]);
    if (hipEventQuery(e) == hipSuccess) {
      (void)hipEventDestroy(e);
      P.free.emplace_back(std::get<1>(P.waiting[i]), std::get<2>(P.waiting[i]));
      P.waiting[i] = P.waiting.back();
      P.waiting.pop_back();
    } else {
      ++i;
    }
  }
  (void)hipGetLastError();            // hipEventQuery's not-ready status
  if (P.free.empty()) {
    unsigned* h = nullptr;
    unsigned* d = nullptr;
    if (hipHostMalloc(reinterpret_cast<void**>(&h), (size_t)FB_CHUNK_SLOTS * FB_SLOT_WORDS * sizeof(unsigned),
                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
        hipHostGetDevicePointer(reinterpret_cast<void**>(&d), h, 0) != hipSuccess) {
      (void)hipGetLastError();
      if (h) (void)hipHostFree(h);
      return false;
    }
    for (int k = FB_CHUNK_SLOTS - 1; k >= 0; --k)
      P.free.emplace_back(h + k * FB_SLOT_WORDS, d + k * FB_SLOT_WORDS);
  }
  *host = P.free.back().first;
  *dev = P.free.back().second;
  P.free.pop_back();
  std::memset(*host, 0, FB_SLOT_WORDS * sizeof(unsigned));
  return true;
}

// give a slot back: at once if no queued work can still write it (wait =
// false), else behind an event on the stream (a synchronisation if the
// event cannot be made)
void fb_release(int device, unsigned* host, unsigned* dev, hipStream_t stream, bool pending) {
  FbPool& P = fb_pool(device);
  hipEvent_t e = nullptr;
  if (pending) {
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(e, stream) != hipSuccess) {
      (void)hipGetLastError();
      if (e) (void)hipEventDestroy(e);
      e = nullptr;
      (void)hipStreamSynchronize(stream);
    }
  }
  std::lock_guard<std::mutex> lk(P.mu);
  if (e) P.waiting.emplace_back(e, host, dev);
  else P.free.emplace_back(host, dev);
}

// the state's non-zero initial fields, after the memset (no host staging,
// so creating a handle does not wait for the stream)
__global__ void k_init_state(DevState* st, double tol, unsigned* mirror, int general) {
  if (threadIdx.x == 0) {
    st->tol = tol;
    st->smirror = mirror;
    st->general = general;
  }
}

}  // namespace

// ---- plans: a fixed batched step, launchable without host staging ----

struct odmd_plan_s {
  int device = 0;
  hipStream_t stream = nullptr;
  std::vector<odmd_t> hs;
  void* dev = nullptr;          // PassDesc table, then the CoreArgs and GramArgs tables
  size_t pass_bytes = 0, core_bytes = 0;
  int ngram = 0, gblocks = 0;   // Gram kernels of the BF16 handles
  struct Launch { int first, nd, nblocks, threads, rows2, basis, rb; };
  std::vector<Launch> launches;
  int nside = 0;
  hipStream_t side[NSIDE] = {};
  hipEvent_t fork = nullptr, join[NSIDE] = {};
};

static void plan_free(odmd_plan_t p) {
  for (int i = 0; i < NSIDE; ++i) {
    if (p->side[i]) (void)hipStreamDestroy(p->side[i]);
    if (p->join[i]) (void)hipEventDestroy(p->join[i]);
  }
  if (p->fork) (void)hipEventDestroy(p->fork);
  if (p->dev) (void)hipFree(p->dev);
  (void)hipGetLastError();
  for (odmd_t h : p->hs) --h->plans;
  delete p;
}


extern "C" {

const char* odmd_status_str(odmd_status s) {
  switch (s) {
    case ODMD_OK: return "ok";
    case ODMD_EINVAL: return "invalid argument";
    case ODMD_ENOMEM: return "out of device memory or workspace too small";
    case ODMD_EEMPTY: return "model has rank 0";
    case ODMD_ENONFINITE: return "non-finite snapshot (update skipped)";
    case ODMD_ENOCONV: return "iteration cap reached";
    case ODMD_ESEQ: return "snapshot pair does not chain (update skipped)";
    case ODMD_EDEVICE: return "HIP device error";
  }
  return "unknown status";
}

size_t odmd_state_bytes(int64_t n, int32_t r_max, odmd_dtype basis, odmd_dtype io) {
  if (!valid_args(n, r_max, 0.0, basis, io)) return 0;
  return make_layout(n, r_max, basis, false, default_shape(n)).total;
}

size_t odmd_state_bytes_general(int64_t n, int32_t r_max, odmd_dtype basis, odmd_dtype io) {
  if (!valid_args(n, r_max, 0.0, basis, io)) return 0;
  return make_layout(n, r_max, basis, true, default_shape(n)).total;
}

size_t odmd_state_bytes_shaped(int64_t n, int32_t r_max, odmd_dtype basis, odmd_dtype io,
                               int32_t threads, int32_t rows_per_block, int32_t max_blocks,
                               int32_t general) {
  const PassShape sh = {threads, rows_per_block, max_blocks};
  if (!valid_args(n, r_max, 0.0, basis, io) || !valid_shape(sh) || (general != 0 && general != 1))
    return 0;
  return make_layout(n, r_max, basis, general != 0, sh).total;
}

odmd_status odmd_default_shape(int64_t n, int32_t* threads, int32_t* rows_per_block,
                               int32_t* max_blocks) {
  if (n < 1 || !threads || !rows_per_block || !max_blocks) return ODMD_EINVAL;
  const PassShape sh = default_shape(n);
  *threads = sh.threads;
  *rows_per_block = sh.rows_per_block;
  *max_blocks = sh.max_blocks;
  return ODMD_OK;
}

static odmd_status create_impl(int64_t n, int32_t r_max, double tol, odmd_dtype basis,
                               odmd_dtype io, void* hip_stream, void* workspace,
                               size_t workspace_bytes, bool general, const PassShape& sh,
                               odmd_t* h) {
  if (!h) return ODMD_EINVAL;
  *h = nullptr;
  if (!valid_args(n, r_max, tol, basis, io) || !valid_shape(sh)) return ODMD_EINVAL;
  const Layout L = make_layout(n, r_max, basis, general, sh);
  if (workspace) {
    if (workspace_bytes < L.total) return ODMD_ENOMEM;
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return ODMD_EINVAL;
  } else if (workspace_bytes != 0) {
    return ODMD_EINVAL;
  }
  odmd_s* s = new (std::nothrow) odmd_s;
  if (!s) return ODMD_ENOMEM;
  s->n = n;
  s->r_max = r_max;
  s->ct = L.ct;
  s->tol = tol;
  // FP64 and FP32 bases take the tolerance as given (the refold is FP64, so
  // FP32 storage adds only its own rounding to the new columns).  A BF16
  // basis is re-orthonormalised after each refold (Gram kernel), but the
  // span of the rounded columns still differs from the basis by about 2^-9:
  // the next snapshots show that difference as residuals of about 1e-3 of
  // their norm, and a tolerance of 2^-12 lets truncation drop those again.
  s->tol_eff = basis == ODMD_BF16 ? std::max(tol, 0x1p-12) : tol;
  s->basis = basis;
  s->io = io;
  s->stream = static_cast<hipStream_t>(hip_stream);
  s->nblk = L.nblk;
  s->threads = L.threads;
  s->rows2 = wide_rows(basis, L.threads, n);
  s->units = L.units;
  {
    const char* alg = std::getenv("ODMD_CORE_SVD");
    s->jacobi_only = alg && std::strcmp(alg, "jacobi") == 0;
  }
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return ODMD_EDEVICE;
  }
  // word 0: the rank feedback, word 1: host-visible copy of the latched status
  if (!fb_acquire(s->device, &s->fb_host, &s->fb_dev)) {
    delete s;
    return ODMD_ENOMEM;
  }
  if (workspace) {
    s->mem = static_cast<char*>(workspace);
  } else {
    if (hipMalloc(&s->mem, L.total) != hipSuccess) {
      (void)hipGetLastError();
      fb_release(s->device, s->fb_host, s->fb_dev, s->stream, false);
      delete s;
      return ODMD_ENOMEM;
    }
    s->own = true;
  }
  s->bytes = L.total;
  if (basis == ODMD_BF16) {
    s->grec = reinterpret_cast<double*>(s->mem + L.gram);
    s->gnwg = L.gnwg;
  }
  s->st = reinterpret_cast<DevState*>(s->mem + L.st);
  s->partials = reinterpret_cast<double*>(s->mem + L.partials);
  s->Us = s->mem + L.Us;
  s->general = general;
  if (general) {
    s->tst = reinterpret_cast<DevState*>(s->mem + L.tst);
    s->pproj = reinterpret_cast<double*>(s->mem + L.pproj);
    s->pt = reinterpret_cast<double*>(s->mem + L.pt);
    s->Ts = s->mem + L.Ts;
    s->eout = s->mem + L.eout;
  }
  // zero state, then its non-zero fields, in the stream's order: the first
  // update on the stream sees them; nothing here waits for the stream
  if (hipMemsetAsync(s->mem, 0, L.total, s->stream) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize(s->stream);
    if (s->own) (void)hipFree(s->mem);
    fb_release(s->device, s->fb_host, s->fb_dev, s->stream, false);
    delete s;
    return ODMD_EDEVICE;
  }
  hipLaunchKernelGGL(k_init_state, dim3(1), dim3(64), 0, s->stream, s->st, s->tol_eff, s->fb_dev + 1,
                     general ? 1 : 0);
  if (hipGetLastError() != hipSuccess) {
    (void)hipStreamSynchronize(s->stream);
    if (s->own) (void)hipFree(s->mem);
    fb_release(s->device, s->fb_host, s->fb_dev, s->stream, false);
    delete s;
    return ODMD_EDEVICE;
  }
  *h = s;
  return ODMD_OK;
}

odmd_status odmd_create_ex(int64_t n, int32_t r_max, double tol, odmd_dtype basis, odmd_dtype io,
                           void* hip_stream, void* workspace, size_t workspace_bytes, odmd_t* h) {
  return create_impl(n, r_max, tol, basis, io, hip_stream, workspace, workspace_bytes, false,
                     default_shape(n), h);
}

odmd_status odmd_create_general(int64_t n, int32_t r_max, double tol, odmd_dtype basis,
                                odmd_dtype io, void* hip_stream, void* workspace,
                                size_t workspace_bytes, odmd_t* h) {
  return create_impl(n, r_max, tol, basis, io, hip_stream, workspace, workspace_bytes, true,
                     default_shape(n), h);
}

odmd_status odmd_create_shaped(int64_t n, int32_t r_max, double tol, odmd_dtype basis,
                               odmd_dtype io, void* hip_stream, int32_t threads,
                               int32_t rows_per_block, int32_t max_blocks, int32_t general,
                               void* workspace, size_t workspace_bytes, odmd_t* h) {
  if (h) *h = nullptr;
  if (general != 0 && general != 1) return ODMD_EINVAL;
  return create_impl(n, r_max, tol, basis, io, hip_stream, workspace, workspace_bytes,
                     general != 0, PassShape{threads, rows_per_block, max_blocks}, h);
}

odmd_status odmd_create(int64_t n, int32_t r_max, double tol, odmd_t* h) {
  return odmd_create_ex(n, r_max, tol, ODMD_F64, ODMD_F64, nullptr, nullptr, 0, h);
}

odmd_status odmd_update(odmd_t h, const void* x_k, const void* x_k1) {
  if (!h || !x_k || !x_k1) return ODMD_EINVAL;
  HIP_OK(hipSetDevice(h->device));
  return launch_update(h, x_k, x_k1);
}

odmd_status odmd_update_batch(odmd_t* hs, const void* const* xs, const void* const* ys,
                              int32_t count) {
  if (!hs || !xs || !ys || count < 0) return ODMD_EINVAL;
  if (count == 0) return ODMD_OK;
  std::unordered_set<odmd_t> seen;
  for (int32_t i = 0; i < count; ++i) {
    if (!hs[i] || !xs[i] || !ys[i] || hs[i]->general) return ODMD_EINVAL;
    if (hs[i]->stream != hs[0]->stream || hs[i]->device != hs[0]->device) return ODMD_EINVAL;
    if (!seen.insert(hs[i]).second) return ODMD_EINVAL;
  }
  HIP_OK(hipSetDevice(hs[0]->device));
  if (capturing(hs[0]->stream)) return ODMD_EINVAL;   // staged through host memory: use a plan
  return launch_batch(hs, xs, ys, count);
}

odmd_status odmd_update_batch_noalloc(odmd_t* hs, const void* const* xs, const void* const* ys,
                                      int32_t count) {
  if (!hs || !xs || !ys || count < 0 || count > NOALLOC_MAX) return ODMD_EINVAL;
  if (count == 0) return ODMD_OK;
  for (int32_t i = 0; i < count; ++i) {
    if (!hs[i] || !xs[i] || !ys[i] || hs[i]->general) return ODMD_EINVAL;
    if (hs[i]->stream != hs[0]->stream || hs[i]->device != hs[0]->device) return ODMD_EINVAL;
  }
  {
    // duplicates: sorted copy of the handles on the stack (nothing allocated)
    odmd_t sorted[NOALLOC_MAX];
    std::copy(hs, hs + count, sorted);
    std::sort(sorted, sorted + count);
    for (int32_t i = 1; i < count; ++i)
      if (sorted[i] == sorted[i - 1]) return ODMD_EINVAL;
  }
  HIP_OK(hipSetDevice(hs[0]->device));
  if (capturing(hs[0]->stream)) return ODMD_EINVAL;   // the tables are copied from host memory
  return launch_batch_noalloc(hs, xs, ys, count);
}

odmd_status odmd_peek_status(odmd_t h, odmd_status* status) {
  if (!h || !status) return ODMD_EINVAL;
  *status = map_status((int)__atomic_load_n(h->fb_host + 1, __ATOMIC_ACQUIRE));
  return ODMD_OK;
}

odmd_status odmd_sync(odmd_t h) {
  if (!h) return ODMD_EINVAL;
  HIP_OK(hipSetDevice(h->device));
  return sync_and_status(h);
}

odmd_status odmd_eigs(odmd_t h, int32_t cap, int32_t* r, double* lam_re, double* lam_im,
                      double* v_re, double* v_im) {
  if (!h || !r || !lam_re || !lam_im || cap < 0) return ODMD_EINVAL;
  if ((v_re == nullptr) != (v_im == nullptr)) return ODMD_EINVAL;
  HIP_OK(hipSetDevice(h->device));
  HIP_OK(launch_eig(h->st, v_re != nullptr, h->stream));
  int rr = 0;
  std::vector<double> lr(RMAX), li(RMAX), vr, vi;
  odmd_status s;
  if ((s = copy_field(h, &rr, &h->st->r, 1)) != ODMD_OK) return s;
  if ((s = copy_field(h, lr.data(), h->st->lam_re, RMAX)) != ODMD_OK) return s;
  if ((s = copy_field(h, li.data(), h->st->lam_im, RMAX)) != ODMD_OK) return s;
  if (v_re) {
    vr.resize(RMAX * RMAX);
    vi.resize(RMAX * RMAX);
    if ((s = copy_field(h, vr.data(), h->st->V_re, RMAX * RMAX)) != ODMD_OK) return s;
    if ((s = copy_field(h, vi.data(), h->st->V_im, RMAX * RMAX)) != ODMD_OK) return s;
  }
  s = sync_and_status(h);
  *r = rr;
  if (s != ODMD_OK) return s;
  if (rr == 0) return ODMD_EEMPTY;
  if (cap < rr) return ODMD_EINVAL;
  for (int k = 0; k < rr; ++k) {
    lam_re[k] = lr[k];
    lam_im[k] = li[k];
  }
  if (v_re) {
    for (int j = 0; j < rr; ++j)
      for (int i = 0; i < rr; ++i) {
        v_re[j * rr + i] = vr[j * RMAX + i];
        v_im[j * rr + i] = vi[j * RMAX + i];
      }
  }
  return ODMD_OK;
}

odmd_status odmd_predict(odmd_t h, int32_t steps, void* out) {
  if (!h || !out || steps < 1) return ODMD_EINVAL;
  HIP_OK(hipSetDevice(h->device));
  return launch_rollout(h, steps, out);
}

odmd_status odmd_predict_batch(odmd_t* hs, const int32_t* steps, void* const* outs, int32_t count) {
  if (!hs || !steps || !outs || count < 0) return ODMD_EINVAL;
  if (count == 0) return ODMD_OK;
  std::unordered_set<odmd_t> seen;
  for (int32_t i = 0; i < count; ++i) {
    if (!hs[i] || !outs[i] || steps[i] < 1) return ODMD_EINVAL;
    if (hs[i]->stream != hs[0]->stream || hs[i]->device != hs[0]->device) return ODMD_EINVAL;
    if (!seen.insert(hs[i]).second) return ODMD_EINVAL;
  }
  HIP_OK(hipSetDevice(hs[0]->device));
  if (capturing(hs[0]->stream)) return ODMD_EINVAL;   // staged through host memory
  {
    std::unique_lock<std::mutex> lk;
    BatchSlot* sl = nullptr;
    // the states' table, then the first chunk's step counts
    const size_t tb = round_up((int64_t)count * sizeof(DevState*), 16);
    const odmd_status s = acquire_slot(hs[0]->device, tb + (size_t)count * sizeof(int), lk, sl);
    if (s != ODMD_OK) return s;
    DevState** tab = static_cast<DevState**>(sl->host);
    int* ks = reinterpret_cast<int*>(static_cast<char*>(sl->host) + tb);
    for (int32_t i = 0; i < count; ++i) {
      tab[i] = hs[i]->st;
      ks[i] = std::min(coef_chunk(hs[i]->r_max), (int)steps[i]);
    }
    HIP_OK(hipMemcpyAsync(sl->dev, sl->host, tb + (size_t)count * sizeof(int), hipMemcpyHostToDevice,
                          hs[0]->stream));
    HIP_OK(launch_power_coef_batch(static_cast<DevState* const*>(sl->dev),
                                   reinterpret_cast<const int*>(static_cast<char*>(sl->dev) + tb), count,
                                   hs[0]->stream));
    HIP_OK(hipEventRecord(sl->done, hs[0]->stream));
    sl->used = true;
  }
  for (int32_t i = 0; i < count; ++i) {
    const odmd_status s = launch_rollout(hs[i], steps[i], outs[i], true);
    if (s != ODMD_OK) return s;
  }
  return ODMD_OK;
}

odmd_status odmd_get_basis(odmd_t h, double* out) {
  if (!h || !out) return ODMD_EINVAL;
  HIP_OK(hipSetDevice(h->device));
  HIP_OK(launch_basis_coef(h->st, h->stream));
  return launch_combine_cols(h, out, h->n, h->r_max, false);
}

odmd_status odmd_get_info(odmd_t h, odmd_info* info) {
  if (!h || !info) return ODMD_EINVAL;
  HIP_OK(hipSetDevice(h->device));
  DevState hdr;
  const size_t nbytes = offsetof(DevState, pad_);
  HIP_OK(hipMemcpyAsync(&hdr, h->st, nbytes, hipMemcpyDeviceToHost, h->stream));
  HIP_OK(hipStreamSynchronize(h->stream));
  info->r = hdr.r;
  info->r_max = h->r_max;
  info->n = h->n;
  info->m = hdr.m_acc;
  info->tol_eff = h->tol_eff;
  info->last_rho = hdr.last_rho;
  info->last_sweeps = hdr.sweeps;
  info->nblocks = h->nblk;
  info->threads = h->threads;
  info->stored = hdr.m;
  info->capacity = h->ct;
  return ODMD_OK;
}

odmd_status odmd_get_state(odmd_t h, int32_t cap, double* sigma, double* atilde, double* p_y,
                           double* C, double* w) {
  if (!h || cap < 0) return ODMD_EINVAL;
  HIP_OK(hipSetDevice(h->device));
  int rr = 0;
  std::vector<double> sg(RMAX), py(RMAX), ww(RMAX), at(RMAX * RMAX), cc(RMAX * RMAX);
  odmd_status s;
  if ((s = copy_field(h, &rr, &h->st->r, 1)) != ODMD_OK) return s;
  if ((s = copy_field(h, sg.data(), h->st->sigma, RMAX)) != ODMD_OK) return s;
  if ((s = copy_field(h, py.data(), h->st->py, RMAX)) != ODMD_OK) return s;
  if ((s = copy_field(h, ww.data(), h->st->w, RMAX)) != ODMD_OK) return s;
  if ((s = copy_field(h, at.data(), h->st->At, RMAX * RMAX)) != ODMD_OK) return s;
  if ((s = copy_field(h, cc.data(), h->st->C, RMAX * RMAX)) != ODMD_OK) return s;
  HIP_OK(hipStreamSynchronize(h->stream));
  if (cap < rr) return ODMD_EINVAL;
  for (int i = 0; i < rr; ++i) {
    if (sigma) sigma[i] = sg[i];
    if (p_y) p_y[i] = py[i];
    if (w) w[i] = ww[i];
    for (int j = 0; j < rr; ++j) {
      if (atilde) atilde[j * rr + i] = at[j * RMAX + i];
      if (C) C[j * rr + i] = cc[j * RMAX + i];
    }
  }
  return ODMD_OK;
}

odmd_status odmd_profile(odmd_t h, int32_t capacity) {
  if (!h || capacity < 0) return ODMD_EINVAL;
  HIP_OK(hipSetDevice(h->device));
  while (h->ev.size() < EV_PER_UPDATE * (size_t)capacity) {
    hipEvent_t e;
    HIP_OK(hipEventCreate(&e));
    h->ev.push_back(e);
  }
  h->prof = capacity > 0;
  return ODMD_OK;
}

// durations of timed update k: pass, core (NaN for a latency-only update),
// and pass start to core end
static odmd_status update_times(odmd_t h, size_t k, float* t) {
  const hipEvent_t* e = &h->ev[EV_PER_UPDATE * k];
  if (k < h->ev_lat.size() && h->ev_lat[k]) {
    t[0] = t[1] = NAN;
  } else {
    HIP_OK(hipEventElapsedTime(&t[0], e[0], e[1]));
    HIP_OK(hipEventElapsedTime(&t[1], e[2], e[3]));
  }
  HIP_OK(hipEventElapsedTime(&t[2], e[0], e[3]));
  return ODMD_OK;
}

odmd_status odmd_profile_read(odmd_t h, double* pass_ms, double* core_ms, int64_t* count) {
  if (!h || !pass_ms || !core_ms || !count) return ODMD_EINVAL;
  HIP_OK(hipSetDevice(h->device));
  HIP_OK(hipStreamSynchronize(h->stream));
  const size_t n = h->ev_used / EV_PER_UPDATE;
  double a = 0.0, b = 0.0;
  int64_t nk = 0;
  for (size_t k = 0; k < n; ++k) {
    float t[3];
    const odmd_status st = update_times(h, k, t);
    if (st != ODMD_OK) return st;
    if (t[0] == t[0]) {
      a += t[0];
      b += t[1];
      ++nk;
    }
  }
  *pass_ms = a;
  *core_ms = b;
  *count = nk;
  h->ev_used = 0;
  h->ev_lat.clear();
  return ODMD_OK;
}

odmd_status odmd_profile_latency(odmd_t h, int32_t on) {
  if (!h) return ODMD_EINVAL;
  h->prof_lat = on != 0;
  return ODMD_OK;
}

odmd_status odmd_profile_samples(odmd_t h, int64_t cap, double* pass_ms, double* core_ms,
                                 double* update_ms, int64_t* count) {
  if (!h || !pass_ms || !core_ms || !count || cap < 0) return ODMD_EINVAL;
  HIP_OK(hipSetDevice(h->device));
  HIP_OK(hipStreamSynchronize(h->stream));
  const int64_t n = (int64_t)(h->ev_used / EV_PER_UPDATE);
  for (int64_t k = 0; k < n && k < cap; ++k) {
    float t[3];
    const odmd_status st = update_times(h, (size_t)k, t);
    if (st != ODMD_OK) return st;
    pass_ms[k] = t[0];
    core_ms[k] = t[1];
    if (update_ms) update_ms[k] = t[2];
  }
  *count = n;
  h->ev_used = 0;
  h->ev_lat.clear();
  return ODMD_OK;
}

odmd_status odmd_destroy(odmd_t h) {
  if (!h || h->plans > 0) return ODMD_EINVAL;
  odmd_status s = ODMD_OK;
  if (hipSetDevice(h->device) != hipSuccess || hipStreamSynchronize(h->stream) != hipSuccess)
    s = ODMD_EDEVICE;
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  if (h->own && hipFree(h->mem) != hipSuccess) s = ODMD_EDEVICE;
  fb_release(h->device, h->fb_host, h->fb_dev, h->stream, false);
  (void)hipGetLastError();
  delete h;
  return s;
}

odmd_status odmd_release(odmd_t h) {
  if (!h || h->plans > 0) return ODMD_EINVAL;
  if (h->own) return odmd_destroy(h);     // freeing its memory waits anyway
  odmd_status s = ODMD_OK;
  if (hipSetDevice(h->device) != hipSuccess) s = ODMD_EDEVICE;
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  fb_release(h->device, h->fb_host, h->fb_dev, h->stream, true);
  (void)hipGetLastError();
  delete h;
  return s;
}

odmd_status odmd_plan_create(odmd_t* hs, const void* const* xs, const void* const* ys,
                             int32_t count, odmd_plan_t* plan) {
  if (!plan) return ODMD_EINVAL;
  *plan = nullptr;
  if (!hs || !xs || !ys || count < 1) return ODMD_EINVAL;
  std::unordered_set<odmd_t> seen;
  for (int32_t i = 0; i < count; ++i) {
    if (!hs[i] || !xs[i] || !ys[i] || hs[i]->general) return ODMD_EINVAL;
    if (hs[i]->stream != hs[0]->stream || hs[i]->device != hs[0]->device) return ODMD_EINVAL;
    if (!seen.insert(hs[i]).second) return ODMD_EINVAL;
  }
  HIP_OK(hipSetDevice(hs[0]->device));
  odmd_plan_s* p = new (std::nothrow) odmd_plan_s;
  if (!p) return ODMD_ENOMEM;
  p->device = hs[0]->device;
  p->stream = hs[0]->stream;
  // grouped like a batched update by (launch shape, rows per lane, storage
  // type, capacity); each workgroup chooses its live-column variant on the
  // device from the stream's m (the host cannot follow m across replays)
  std::map<std::tuple<int, int, int, int>, std::vector<int32_t>> groups;
  for (int32_t i = 0; i < count; ++i)
    groups[{hs[i]->threads, hs[i]->rows2, (int)hs[i]->basis, hs[i]->ct}].push_back(i);
  p->pass_bytes = round_up((int64_t)count * sizeof(PassDesc), 256);
  p->core_bytes = round_up((int64_t)count * sizeof(CoreArgs), 256);
  const size_t bytes = p->pass_bytes + p->core_bytes + (size_t)count * sizeof(GramArgs);
  std::vector<char> host(bytes, 0);
  PassDesc* pd = reinterpret_cast<PassDesc*>(host.data());
  CoreArgs* cd = reinterpret_cast<CoreArgs*>(host.data() + p->pass_bytes);
  p->ngram = fill_gram(hs, count, reinterpret_cast<GramArgs*>(host.data() + p->pass_bytes + p->core_bytes),
                       &p->gblocks);
  int k = 0;
  for (auto& g : groups) {
    std::stable_sort(g.second.begin(), g.second.end(), [&](int32_t a, int32_t b) {
      return hs[a]->n * hs[b]->nblk > hs[b]->n * hs[a]->nblk;
    });
    odmd_plan_s::Launch L{k, 0, 0, std::get<0>(g.first), std::get<1>(g.first), std::get<2>(g.first),
                          std::get<3>(g.first)};
    for (int32_t i : g.second) {
      odmd_t h = hs[i];
      PassDesc& d = pd[k++];
      d = PassDesc{};
      d.Us = h->Us;
      d.x = xs[i];
      d.y = ys[i];
      d.partials = h->partials;
      d.st = h->st;
      d.n = h->n;
      d.nblk = h->nblk;
      d.ct = h->ct;
      d.blk0 = L.nblocks;
      L.nblocks += h->nblk;
      ++L.nd;
    }
    p->launches.push_back(L);
  }
  for (int32_t i = 0; i < count; ++i) {
    odmd_t h = hs[i];
    CoreArgs& c = cd[i];
    c = CoreArgs{};   // fb stays null: a plan step reports nothing to the host
    c.st = h->st;
    c.partials = h->partials;
    c.nblk = h->nblk;
    c.r_max = h->r_max;
    c.jacobi_only = h->jacobi_only;
    c.rb = -h->ct;        // the pass's variant follows m on the device
    c.ct = h->ct;
    c.fold_slack = fold_slack(h);
    c.grec = h->grec;
    c.gnwg = h->gnwg;
  }
  p->nside = p->launches.size() > 1 ? std::min<int>(NSIDE, (int)p->launches.size()) : 0;
  bool ok = hipMalloc(&p->dev, bytes) == hipSuccess &&
            hipMemcpy(p->dev, host.data(), bytes, hipMemcpyHostToDevice) == hipSuccess;
  if (ok && p->nside > 0) {
    ok = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; ok && i < p->nside; ++i)
      ok = hipStreamCreateWithFlags(&p->side[i], hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&p->join[i], hipEventDisableTiming) == hipSuccess;
  }
  if (!ok) {
    plan_free(p);
    return ODMD_ENOMEM;
  }
  for (int32_t i = 0; i < count; ++i) {
    hs[i]->full_bucket = true;
    ++hs[i]->plans;
    p->hs.push_back(hs[i]);
  }
  *plan = p;
  return ODMD_OK;
}

odmd_status odmd_plan_launch(odmd_plan_t p) {
  if (!p) return ODMD_EINVAL;
  HIP_OK(hipSetDevice(p->device));
  const PassDesc* dpd = static_cast<const PassDesc*>(p->dev);
  if (p->nside == 0) {
    const odmd_plan_s::Launch& L = p->launches[0];
    HIP_OK(launch_pass_batch_live(dpd + L.first, L.nd, L.nblocks, L.threads, L.rows2, L.basis, L.rb,
                                  p->stream));
  } else {
    HIP_OK(hipEventRecord(p->fork, p->stream));
    for (int i = 0; i < p->nside; ++i) HIP_OK(hipStreamWaitEvent(p->side[i], p->fork, 0));
    for (size_t i = 0; i < p->launches.size(); ++i) {
      const odmd_plan_s::Launch& L = p->launches[i];
      HIP_OK(launch_pass_batch_live(dpd + L.first, L.nd, L.nblocks, L.threads, L.rows2, L.basis, L.rb,
                                    p->side[i % p->nside]));
    }
    for (int i = 0; i < p->nside; ++i) {
      HIP_OK(hipEventRecord(p->join[i], p->side[i]));
      HIP_OK(hipStreamWaitEvent(p->stream, p->join[i], 0));
    }
  }
  if (p->ngram > 0)
    HIP_OK(launch_gram_batch(reinterpret_cast<const GramArgs*>(static_cast<char*>(p->dev) + p->pass_bytes +
                                                               p->core_bytes),
                             p->ngram, p->gblocks, p->stream));
  HIP_OK(launch_core_batch(
      reinterpret_cast<const CoreArgs*>(static_cast<char*>(p->dev) + p->pass_bytes),
      (int)p->hs.size(), p->stream));
  return ODMD_OK;
}

odmd_status odmd_plan_destroy(odmd_plan_t p) {
  if (!p) return ODMD_EINVAL;
  odmd_status s = ODMD_OK;
  if (hipSetDevice(p->device) != hipSuccess || hipStreamSynchronize(p->stream) != hipSuccess)
    s = ODMD_EDEVICE;
  plan_free(p);
  return s;
}

}  // extern "C"
