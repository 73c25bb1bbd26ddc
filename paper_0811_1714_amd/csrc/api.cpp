// C-ABI entry points: argument validation, schedule resolution, workspace, and the
// Strassen-Winograd executor (Section 4, Algorithm 4) over the base-case kernels.
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "gf2_internal.h"

namespace gf2 {

// ---------------------------------------------------------------- errors
namespace {
thread_local char g_err[512] = "";
}

gf2_status set_error(gf2_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return s;
}

gf2_status hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return GF2_OK;
  return set_error(GF2_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ---------------------------------------------------------------- workspace
namespace {

constexpr int kMaxDevices = 64;

struct DeviceState {
  std::mutex mu;
  void* base = nullptr;
  size_t bytes = 0;
  hipEvent_t last = nullptr;   // recorded after the last enqueued use
  hipStream_t last_stream = nullptr;
  bool has_last = false;
  // A graph captured while using ``base`` keeps its address and may be replayed at any time,
  // so such a buffer is never freed before gf2_shutdown: growing past it allocates a new
  // buffer and keeps the old one here.
  bool captured = false;
  std::vector<void*> retired;
};
DeviceState g_dev[kMaxDevices];

bool fault_alloc() {
  const char* e = getenv("GF2_FAULT_ALLOC");
  return e && e[0] == '1';
}

// Holds the device's workspace for the duration of one call: waits for the previous
// user on another stream, and on release records an event so the next user waits.
class WorkspaceLease {
 public:
  WorkspaceLease() = default;
  ~WorkspaceLease() { release(); }
  gf2_status acquire(size_t need, hipStream_t s) {
    int dev = 0;
    gf2_status st = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (st != GF2_OK) return st;
    if (dev < 0 || dev >= kMaxDevices) return set_error(GF2_ERR_UNSUPPORTED, "device id %d out of range", dev);
    ds_ = &g_dev[dev];
    ds_->mu.lock();
    locked_ = true;
    stream_ = s;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    st = hip_check(hipStreamIsCapturing(s, &cs), "hipStreamIsCapturing");
    if (st != GF2_OK) return st;
    const bool capturing = cs != hipStreamCaptureStatusNone;
    if (need > ds_->bytes) {
      if (capturing)
        return set_error(GF2_ERR_CAPTURE, "needs %zu bytes of workspace under stream capture; call "
                         "gf2_reserve_workspace first", need);
      if (fault_alloc()) return set_error(GF2_ERR_ALLOC, "injected allocation failure (GF2_FAULT_ALLOC)");
      st = hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
      if (st != GF2_OK) return st;
      const size_t grow = need + need / 4 + (1u << 20);
      void* fresh = nullptr;
      if (hipMalloc(&fresh, grow) != hipSuccess)
        return set_error(GF2_ERR_ALLOC, "hipMalloc of %zu bytes of workspace failed", grow);
      if (ds_->base) {
        if (ds_->captured) ds_->retired.push_back(ds_->base);
        else (void)hipFree(ds_->base);
      }
      ds_->base = fresh;
      ds_->bytes = grow;
      ds_->captured = false;
    }
    if (capturing && need > 0) ds_->captured = true;
    if (!ds_->last) {
      st = hip_check(hipEventCreateWithFlags(&ds_->last, hipEventDisableTiming), "hipEventCreate");
      if (st != GF2_OK) return st;
    }
    if (ds_->has_last && ds_->last_stream != s) {
      st = hip_check(hipStreamWaitEvent(s, ds_->last, 0), "hipStreamWaitEvent");
      if (st != GF2_OK) return st;
    }
    return GF2_OK;
  }
  void* ptr() const { return ds_ ? ds_->base : nullptr; }
  void used() { used_ = true; }
  void release() {
    if (!locked_) return;
    if (used_ && ds_->last && hipEventRecord(ds_->last, stream_) == hipSuccess) {
      ds_->has_last = true;
      ds_->last_stream = stream_;
    }
    ds_->mu.unlock();
    locked_ = false;
  }

 private:
  DeviceState* ds_ = nullptr;
  bool locked_ = false, used_ = false;
  hipStream_t stream_ = nullptr;
};

// ---------------------------------------------------------------- schedule
std::mutex g_sched_mu;
bool g_has_override = false;
gf2_schedule g_override{};

uint64_t tail_of(int64_t cols) { return (cols & 63) ? ((1ull << (cols & 63)) - 1) : ~0ull; }

// M4RM table width of a schedule (0 in a schedule means 8).
inline int kappa_of(const gf2_schedule& s) { return s.kappa > 0 ? s.kappa : 8; }


bool splittable(int64_t m, int64_t k, int64_t n, int64_t cutoff);

int compute_units() {
  static std::atomic<int> cached{0};
  int c = cached.load();
  if (c == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
      c = 256;
    cached.store(c);
  }
  return c;
}

// Predicted time (ms) of an M4RM schedule on MI355X, fitted to 2935 timed schedules on 71
// shapes: 22 from 1024^3 to 32768^3 and rectangles down to n = 129 (every tile the default
// chooses from, k split and Strassen-Winograd depth), 65536^3 on the tallest tiles, and 48
// products below 2^30 bit-operations with m, k, n log-uniform in [64, 4096).  The fit weights
// each shape's schedules within 15% of its fastest six-fold.  The schedule it picks is 1.4%
// slower than the fastest on the small products and 3.8% on the large ones (leave-one-shape-
// out, before the 65536^3 timings were added: 1.4% and 4.0%).
//   * tiles run in rounds of one per compute unit; a Strassen leaf launch whose last round
//     is at most half full spreads that round's work over all units (``run_leaves``);
//   * a tile costs, per tile family (rows of B per barrier phase), a fixed start-up, a
//     cost per phase (table build, barrier, B loads) and a cost per tile row per phase
//     (lookups); see ``kFamily``;
//   * operand traffic (A once per column tile, B once per row tile) at 49 TB/s (mostly
//     cache hits), Strassen passes ((2mk + 2kn + 2.75mn)/8 bytes per node) at 2.5 TB/s, and
//     a k split's zeroing at 0.9 TB/s plus its atomic XORs at 1.0 TB/s.
struct CostFamily {
  int phase_rows;
  double tile_ms, phase_ms, row_phase_ms;
};
constexpr CostFamily kFamily[] = {
    {16, 1.169e-2, 5.16e-4, 6.578e-7},    // two tables per 16-row phase, 1024 columns
    {32, 1.459e-2, 5.43e-4, 5.248e-7},    // four tables per 32-row phase, 512 columns
    {64, 1.159e-2, 5.741e-4, 9.41e-7},    // eight tables per 64-row phase, 256 columns
    {256, 1.203e-2, 2.473e-3, 1.527e-6},  // 32 tables per 256-row phase, 64 columns
};
constexpr double kAddBytesPerMs = 2.456e9, kOperandBytesPerMs = 4.943e10, kZeroBytesPerMs = 9.091e8,
                 kAtomicBytesPerMs = 9.728e8;

const CostFamily& cost_family(int64_t phase_rows) {
  for (const CostFamily& f : kFamily)
    if (f.phase_rows == phase_rows) return f;
  return kFamily[0];   // single-table tiles (not among the default's choices)
}

struct CostAcc {
  double tile_ms = 0, add_bytes = 0, operand_bytes = 0, zero_bytes = 0, atomic_bytes = 0;
  int64_t tiles = 0, leaves = 0;
};

// ``sk`` > 1 (no recursion): k in sk slices, each a tile of its own, XOR-ed atomically into
// a zeroed C.
void cost_walk(int64_t m, int64_t k, int64_t n, int64_t cutoff, int v, CostAcc& a, int sk = 1) {
  if (!splittable(m, k, n, cutoff)) {
    const int64_t bm = m4rm_tile_rows(v), tw = m4rm_tile_words(v), pr = m4rm_phase_rows(v);
    const CostFamily& f = cost_family(pr);
    const int64_t rt = (m + bm - 1) / bm, ct = (words(n) + tw - 1) / tw, t = rt * ct * sk;
    const int64_t ks = sk > 1 ? std::min<int64_t>(k, 64 * ((words(k) + sk - 1) / sk)) : k;
    a.tiles += t;
    a.leaves += 1;
    a.tile_ms += (double)t * (f.tile_ms + (double)((ks + pr - 1) / pr) * (f.phase_ms + f.row_phase_ms * (double)bm));
    a.operand_bytes += 8.0 * ((double)m * words(k) * ct + (double)k * words(n) * rt);
    if (sk > 1) {
      const double cbytes = 8.0 * (double)m * (double)words(n);
      a.zero_bytes += cbytes;
      a.atomic_bytes += cbytes * sk;
    }
    return;
  }
  a.add_bytes += (2.0 * m * k + 2.0 * k * n + 2.75 * m * n) / 8.0;
  const int64_t m0 = (m + 1) / 2, m1 = m - m0;
  const int64_t k0 = 64 * ((words(k) + 1) / 2), k1 = k - k0;
  const int64_t n0 = 64 * ((words(n) + 1) / 2), n1 = n - n0;
  cost_walk(m0, k0, n0, cutoff, v, a);   // P0, P4, P5, P6
  cost_walk(m0, k0, n0, cutoff, v, a);
  cost_walk(m0, k0, n0, cutoff, v, a);
  cost_walk(m0, k0, n0, cutoff, v, a);
  cost_walk(m0, k1, n0, cutoff, v, a);   // P1
  cost_walk(m0, k1, n1, cutoff, v, a);   // P2
  cost_walk(m1, k1, n0, cutoff, v, a);   // P3
}

double predicted_ms(int64_t m, int64_t k, int64_t n, int64_t cutoff, int v, int sk = 1) {
  CostAcc a;
  cost_walk(m, k, n, cutoff, v, a, sk);
  if (a.tiles == 0) return 0;
  const int64_t cus = compute_units();
  const int64_t full = (a.tiles + cus - 1) / cus, tail = a.tiles - (full - 1) * cus;
  const bool spread = full >= 2 && 2 * tail <= cus && a.leaves >= 2 && a.leaves <= kMaxGroup;
  const double rounds = spread ? (double)(full - 1) + (double)tail / (double)cus : (double)full;
  return rounds * a.tile_ms / (double)a.tiles + a.add_bytes / kAddBytesPerMs + a.operand_bytes / kOperandBytesPerMs +
         a.zero_bytes / kZeroBytesPerMs + a.atomic_bytes / kAtomicBytesPerMs;
}

// Default schedule for a shape (used when no model, tuning result or request says
// otherwise): products with at most eight columns of B take the streamed popcount; all
// others the M4RM tile, Strassen-Winograd depth and k split of lowest predicted time.  A
// k slice keeps at least four words (256 rows) of k.  Results are memoised per shape.
gf2_schedule default_schedule_uncached(int64_t m, int64_t k, int64_t n) {
  gf2_schedule s{};
  s.kernel = GF2_KERNEL_M4RM;
  s.splitk = 1;
  // At most eight columns of B: the popcount base case streams A once against B's columns
  // in LDS (bound by reading A from HBM), ahead of any table method.
  if (cubic_narrow_shape(k, n)) {
    s.kernel = GF2_KERNEL_CUBIC;
    return s;
  }
  const int64_t mn = m < n ? (m < k ? m : k) : (n < k ? n : k);
  double best = -1;
  for (int64_t cutoff : {int64_t(0), mn / 2, mn / 4, mn / 8}) {
    if (cutoff && cutoff < 2048) continue;
    const bool recurse = cutoff > 0 && splittable(m, k, n, cutoff);
    for (int v : {0, 10, 1, 2, 3, 4, 11, 12, 13, 14, 15, 16, 17, 18}) {
      if (v >= m4rm_num_variants()) continue;
      for (int sk : {1, 2, 4, 8, 16, 32}) {
        if (sk > 1 && (recurse || words(k) / sk < 4)) continue;
        const double t = predicted_ms(m, k, n, cutoff, v, sk);
        if (best < 0 || t < best) {
          best = t;
          s.variant = v;
          s.cutoff = (int32_t)cutoff;
          s.splitk = sk;
        }
      }
    }
  }
  return s;
}

gf2_schedule default_schedule(int64_t m, int64_t k, int64_t n) {
  static std::mutex mu;
  static std::map<std::array<int64_t, 3>, gf2_schedule> memo;
  const std::array<int64_t, 3> key{m, k, n};
  {
    std::lock_guard<std::mutex> g(mu);
    auto it = memo.find(key);
    if (it != memo.end()) return it->second;
  }
  const gf2_schedule s = default_schedule_uncached(m, k, n);
  std::lock_guard<std::mutex> g(mu);
  if (memo.size() >= 4096) memo.clear();
  memo.emplace(key, s);
  return s;
}

// ``may_time`` false: under the autotune policy a shape missing from the cache takes the
// default schedule instead of being timed (no allocation, no synchronisation).
gf2_schedule resolve(const gf2_schedule* req, int64_t m, int64_t k, int64_t n, hipStream_t st, bool may_time = true) {
  gf2_schedule s = default_schedule(m, k, n);
  {
    std::lock_guard<std::mutex> g(g_sched_mu);
    if (!req && g_has_override) req = &g_override;
  }
  if (!req) {
    const int c = choose_candidate(m, k, n, false, st, may_time);
    if (c >= 0) s = candidate(c);
  }
  if (req) {
    if (req->kernel != GF2_KERNEL_AUTO) s.kernel = req->kernel;
    if (req->kernel != GF2_KERNEL_AUTO || req->variant) s.variant = req->variant;
    s.cutoff = req->cutoff;
    if (req->splitk > 0) s.splitk = req->splitk;
    s.odd = req->odd;
    s.kappa = req->kappa;
    s.memory = req->memory;
  }
  if (s.kappa <= 0) s.kappa = 8;
  return s;
}

// ---------------------------------------------------------------- validation
int64_t extent_bytes(int64_t rows, int64_t ld, int64_t wds) { return ((rows - 1) * ld + wds) * 8; }

bool overlaps(const void* a, int64_t abytes, const void* b, int64_t bbytes) {
  const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
  return a0 < b0 + (uintptr_t)bbytes && b0 < a0 + (uintptr_t)abytes;
}

constexpr int64_t kMaxLd = int64_t(1) << 21;      // kernels use 32-bit offsets within a tile

gf2_status validate(const uint64_t* C, int64_t ldc, const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb,
                    int64_t m, int64_t k, int64_t n) {
  if (m < 0 || k < 0 || n < 0) return set_error(GF2_ERR_INVALID_ARG, "negative dimension (m=%lld k=%lld n=%lld)",
                                                (long long)m, (long long)k, (long long)n);
  if (m == 0 || n == 0) return GF2_OK;
  if (m > INT32_MAX || k > INT32_MAX || n > INT32_MAX)
    return set_error(GF2_ERR_UNSUPPORTED, "dimensions above 2^31-1 are not supported");
  const int64_t Wk = words(k), Wn = words(n);
  if (!C) return set_error(GF2_ERR_INVALID_ARG, "C is NULL");
  if (ldc < Wn) return set_error(GF2_ERR_INVALID_ARG, "ldc=%lld < ceil(n/64)=%lld", (long long)ldc, (long long)Wn);
  if ((uintptr_t)C & 7) return set_error(GF2_ERR_INVALID_ARG, "C is not 8-byte aligned");
  if (ldc > kMaxLd) return set_error(GF2_ERR_UNSUPPORTED, "ldc above 2^21 words");
  if (k == 0) return GF2_OK;
  if (!A || !B) return set_error(GF2_ERR_INVALID_ARG, "A or B is NULL");
  if (lda < Wk) return set_error(GF2_ERR_INVALID_ARG, "lda=%lld < ceil(k/64)=%lld", (long long)lda, (long long)Wk);
  if (ldb < Wn) return set_error(GF2_ERR_INVALID_ARG, "ldb=%lld < ceil(n/64)=%lld", (long long)ldb, (long long)Wn);
  if (((uintptr_t)A & 7) || ((uintptr_t)B & 7)) return set_error(GF2_ERR_INVALID_ARG, "A or B is not 8-byte aligned");
  if (lda > kMaxLd || ldb > kMaxLd) return set_error(GF2_ERR_UNSUPPORTED, "lda or ldb above 2^21 words");
  const int64_t cb = extent_bytes(m, ldc, Wn);
  if (overlaps(C, cb, A, extent_bytes(m, lda, Wk)) || overlaps(C, cb, B, extent_bytes(k, ldb, Wn)))
    return set_error(GF2_ERR_ALIAS, "C overlaps A or B");
  return GF2_OK;
}

gf2_status validate_sched(const gf2_schedule* s) {
  if (!s) return GF2_OK;
  if (s->kernel < GF2_KERNEL_AUTO || s->kernel > GF2_KERNEL_CUBIC)
    return set_error(GF2_ERR_INVALID_ARG, "unknown kernel %d", s->kernel);
  if (s->kernel != GF2_KERNEL_AUTO && gf2_kernel_variants(s->kernel) == 0)
    return set_error(GF2_ERR_UNSUPPORTED, "kernel %d is not available", s->kernel);
  if (s->variant < 0 || (s->kernel != GF2_KERNEL_AUTO && s->variant >= gf2_kernel_variants(s->kernel)))
    return set_error(GF2_ERR_INVALID_ARG, "variant %d out of range", s->variant);
  if (s->cutoff < 0) return set_error(GF2_ERR_INVALID_ARG, "negative cutoff");
  if (s->splitk < 0 || s->splitk > kMaxGroup) return set_error(GF2_ERR_INVALID_ARG, "splitk must be in [0, %d]", kMaxGroup);
  if (s->odd != GF2_ODD_PAD && s->odd != GF2_ODD_PEEL) return set_error(GF2_ERR_INVALID_ARG, "unknown odd-size rule %d", s->odd);
  if (s->kappa != 0 && (s->kappa < 4 || s->kappa > 8))
    return set_error(GF2_ERR_INVALID_ARG, "table width %d outside 4..8", s->kappa);
  if (s->memory != GF2_MEM_FAST && s->memory != GF2_MEM_LOW)
    return set_error(GF2_ERR_INVALID_ARG, "unknown workspace plan %d", s->memory);
  if (s->kernel == GF2_KERNEL_M4RM && s->kappa != 0 && !m4rm_has_kappa(s->variant, s->kappa))
    return set_error(GF2_ERR_UNSUPPORTED, "M4RM variant %d has no %d-bit tables", s->variant, s->kappa);
  return GF2_OK;
}

// A resolved schedule the kernels can run (the M4RM tile offers its table width).
gf2_status check_resolved(const gf2_schedule& s) {
  if (s.kernel == GF2_KERNEL_M4RM && !m4rm_has_kappa(s.variant, kappa_of(s)))
    return set_error(GF2_ERR_UNSUPPORTED, "M4RM variant %d has no %d-bit tables", s.variant, kappa_of(s));
  return GF2_OK;
}

// ---------------------------------------------------------------- execution
struct View {
  const uint64_t* p;
  int64_t ld, rows, cols;
};

MulDesc make_desc(const View& A, const View& B, uint64_t* C, int64_t ldc, int out) {
  MulDesc d;
  d.A = A.p; d.lda = A.ld;
  d.B = B.p; d.ldb = B.ld;
  d.C = C; d.ldc = ldc;
  d.m = (int32_t)A.rows; d.k = (int32_t)A.cols; d.n = (int32_t)B.cols;
  d.out = out;
  return d;
}

// Scratch the base kernel needs beyond the operands (the popcount kernel's B transpose,
// reused leaf after leaf).
size_t base_scratch_words(const gf2_schedule& s, const std::vector<MulDesc>& ds) {
  size_t w = 0;
  if (s.kernel == GF2_KERNEL_CUBIC)       // products run one after another
    for (const MulDesc& d : ds) w = std::max(w, cubic_scratch_words(d));
  if (s.kernel == GF2_KERNEL_MFMA)        // one grouped launch: every product keeps its B transposed
    for (const MulDesc& d : ds) w += transpose_words(d);
  return w;
}

// Base-case products launched together.
gf2_status run_base(const gf2_schedule& s, const std::vector<MulDesc>& ds, uint64_t* scratch, hipStream_t st) {
  if (ds.empty()) return GF2_OK;
  switch (s.kernel) {
    case GF2_KERNEL_MFMA:
      return mfma_launch_group(ds.data(), (int)ds.size(), scratch, st);
    case GF2_KERNEL_CUBIC:
      for (const MulDesc& d : ds) {
        gf2_status r = cubic_launch(d, scratch, st);
        if (r != GF2_OK) return r;
      }
      return GF2_OK;
    case GF2_KERNEL_M4RM:
    default:
      return m4rm_launch_group(ds.data(), (int)ds.size(), s.variant, st, 0, kappa_of(s));
  }
}


struct StrassenPlan {
  std::vector<PreOp> pre;
  std::vector<MulDesc> leaves;
  std::vector<PostOp> post;
  // Peeling fix-ups.  Inner-slice ones (C ^= A[:, k':] B[k':, :]) run after the
  // post-additions of their node's depth, which write the C they add to; peeled rows and
  // columns only need their node's operands and run after the leaves.
  std::vector<std::pair<int, MulDesc>> kfix;
  std::vector<MulDesc> fix;
  size_t ws_words = 0;
};

inline size_t align_words(size_t w) { return (w + 31) & ~size_t(31); }   // 256-byte alignment

bool splittable(int64_t m, int64_t k, int64_t n, int64_t cutoff) {
  const int64_t c = cutoff < 64 ? 64 : cutoff;
  return cutoff > 0 && m > c && k > c && n > c;
}

// Depth-first construction.  A node pushes its pre-additions before recursing and its
// post-additions after, so both lists run in creation order: pre-ops parents first,
// post-ops children first; the leaves run all at once in between.  ``base`` == nullptr
// only sizes the workspace.
// ``no_p``: the node's P0..P6 are not allocated (the fused two-level passes never use them; the
// plan's post-addition records then hold views of null buffers and must not be launched).
void plan_node(StrassenPlan& pl, uint64_t* base, const View& A, const View& B, uint64_t* C, int64_t ldc,
               int out_mode, int64_t cutoff, int odd, int depth = 0, bool no_p = false) {
  const int64_t m = A.rows, k = A.cols, n = B.cols;
  if (!splittable(m, k, n, cutoff)) {
    pl.leaves.push_back(make_desc(A, B, C, ldc, out_mode));
    return;
  }
  if (odd == GF2_ODD_PEEL) {
    // Section 4, peeling: recurse on the largest part that halves exactly on word
    // borders (rows even, k and n multiples of 128) and add the rest without recursion:
    //   C[:m',:n'] = A[:m',:k'] B[:k',:n'] + A[:m',k':] B[k':,:n']
    //   C[:m',n':] = A[:m',:] B[:,n':]        C[m':,:] = A[m':,:] B
    const int64_t me = m & ~int64_t(1), ke = k & ~int64_t(127), ne = n & ~int64_t(127);
    if (me != m || ke != k || ne != n) {
      if (!splittable(me, ke, ne, cutoff)) {
        pl.leaves.push_back(make_desc(A, B, C, ldc, out_mode));
        return;
      }
      plan_node(pl, base, View{A.p, A.ld, me, ke}, View{B.p, B.ld, ke, ne}, C, ldc, out_mode, cutoff, odd, depth);
      if (ke < k)
        pl.kfix.push_back({depth, make_desc(View{A.p + ke / 64, A.ld, me, k - ke}, View{B.p + ke * B.ld, B.ld, k - ke, ne},
                                            C, ldc, OUT_XOR)});
      if (ne < n)
        pl.fix.push_back(make_desc(View{A.p, A.ld, me, k}, View{B.p + ne / 64, B.ld, k, n - ne}, C + ne / 64, ldc,
                                   out_mode));
      if (me < m)
        pl.fix.push_back(make_desc(View{A.p + me * A.ld, A.ld, m - me, k}, B, C + me * ldc, ldc, out_mode));
      return;
    }
  }
  const int64_t m0 = (m + 1) / 2, m1 = m - m0;
  const int64_t k0w = (words(k) + 1) / 2, k0 = 64 * k0w, k1 = k - k0;
  const int64_t n0w = (words(n) + 1) / 2, n0 = 64 * n0w, n1 = n - n0;
  auto alloc = [&](size_t wds) -> uint64_t* {
    uint64_t* p = base ? base + pl.ws_words : nullptr;
    pl.ws_words += align_words(wds);
    return p;
  };
  uint64_t* S[4];
  uint64_t* T[4];
  uint64_t* P[7];
  for (int i = 0; i < 4; ++i) S[i] = alloc((size_t)(m0 * k0w));
  for (int i = 0; i < 4; ++i) T[i] = alloc((size_t)(k0 * n0w));
  for (int i = 0; i < 7; ++i) P[i] = no_p ? nullptr : alloc((size_t)(m0 * n0w));

  PreOp ps;
  ps.kind = 0;
  ps.depth = depth;
  ps.in[0] = QView{A.p, A.ld, m0, k0w, ~0ull};
  ps.in[1] = QView{A.p + k0w, A.ld, m0, words(k1), tail_of(k1)};
  ps.in[2] = QView{A.p + m0 * A.ld, A.ld, m1, k0w, ~0ull};
  ps.in[3] = QView{A.p + m0 * A.ld + k0w, A.ld, m1, words(k1), tail_of(k1)};
  for (int i = 0; i < 4; ++i) ps.out[i] = S[i];
  ps.ldo = k0w; ps.R = m0; ps.Wd = k0w;
  pl.pre.push_back(ps);
  PreOp pt;
  pt.kind = 1;
  pt.depth = depth;
  pt.in[0] = QView{B.p, B.ld, k0, n0w, ~0ull};
  pt.in[1] = QView{B.p + n0w, B.ld, k0, words(n1), tail_of(n1)};
  pt.in[2] = QView{B.p + k0 * B.ld, B.ld, k1, n0w, ~0ull};
  pt.in[3] = QView{B.p + k0 * B.ld + n0w, B.ld, k1, words(n1), tail_of(n1)};
  for (int i = 0; i < 4; ++i) pt.out[i] = T[i];
  pt.ldo = n0w; pt.R = k0; pt.Wd = n0w;
  pl.pre.push_back(pt);

  const View A_NW{A.p, A.ld, m0, k0}, A_NE{A.p + k0w, A.ld, m0, k1}, A_SE{A.p + m0 * A.ld + k0w, A.ld, m1, k1};
  const View B_NW{B.p, B.ld, k0, n0}, B_SW{B.p + k0 * B.ld, B.ld, k1, n0}, B_SE{B.p + k0 * B.ld + n0w, B.ld, k1, n1};
  const View S0{S[0], k0w, m0, k0}, S1{S[1], k0w, m0, k0}, S2{S[2], k0w, m0, k0}, S3{S[3], k0w, m0, k1};
  const View T0{T[0], n0w, k0, n0}, T1{T[1], n0w, k0, n0}, T2{T[2], n0w, k0, n0}, T3{T[3], n0w, k1, n0};
  plan_node(pl, base, A_NW, B_NW, P[0], n0w, OUT_STORE, cutoff, odd, depth + 1);   // P0 = A_NW B_NW
  plan_node(pl, base, A_NE, B_SW, P[1], n0w, OUT_STORE, cutoff, odd, depth + 1);   // P1 = A_NE B_SW
  plan_node(pl, base, S3, B_SE, P[2], n0w, OUT_STORE, cutoff, odd, depth + 1);     // P2 = S3 B_SE
  plan_node(pl, base, A_SE, T3, P[3], n0w, OUT_STORE, cutoff, odd, depth + 1);     // P3 = A_SE T3
  plan_node(pl, base, S0, T0, P[4], n0w, OUT_STORE, cutoff, odd, depth + 1);       // P4 = S0 T0
  plan_node(pl, base, S1, T1, P[5], n0w, OUT_STORE, cutoff, odd, depth + 1);       // P5 = S1 T1
  plan_node(pl, base, S2, T2, P[6], n0w, OUT_STORE, cutoff, odd, depth + 1);       // P6 = S2 T2

  PostOp po;
  for (int i = 0; i < 7; ++i) po.P[i] = P[i];
  po.ldp = n0w;
  po.c[0] = OView{C, ldc, m0, n0w, ~0ull};
  po.c[1] = OView{C + n0w, ldc, m0, words(n1), tail_of(n1)};
  po.c[2] = OView{C + m0 * ldc, ldc, m1, n0w, ~0ull};
  po.c[3] = OView{C + m0 * ldc + n0w, ldc, m1, words(n1), tail_of(n1)};
  po.mode = out_mode;
  po.depth = depth;
  pl.post.push_back(po);
}

// Split-K: slices at word borders, all XORed atomically into C.
void plan_splitk(std::vector<MulDesc>& out, const View& A, const View& B, uint64_t* C, int64_t ldc, int sk) {
  const int64_t kw = words(A.cols);
  if (sk > kw) sk = (int)kw;
  for (int i = 0; i < sk; ++i) {
    const int64_t w0 = kw * i / sk, w1 = kw * (i + 1) / sk;
    if (w1 <= w0) continue;
    const int64_t kk = (w1 * 64 < A.cols ? w1 * 64 : A.cols) - w0 * 64;
    View a{A.p + w0, A.ld, A.rows, kk}, b{B.p + w0 * 64 * B.ld, B.ld, kk, B.cols};
    out.push_back(make_desc(a, b, C, ldc, OUT_ATOMIC));
  }
}

// Peeling fix-ups are thin products (a few rows, columns or k) with long other sides.  On
// the M4RM kernel each gets a tile height that suits its rows and its k cut into slices
// of about 2048 XOR-ed into C, so no tile runs much longer than a leaf tile; a stored
// result has its region zeroed first.
gf2_status run_fixups(const gf2_schedule& s, const std::vector<MulDesc>& ds, uint64_t* scratch, hipStream_t st) {
  if (ds.empty()) return GF2_OK;
  // Narrow tables read A's index expansion, which a k slice cannot take apart: launch as planned.
  if (s.kernel != GF2_KERNEL_M4RM || kappa_of(s) < 8) return run_base(s, ds, scratch, st);
  gf2_status r;
  std::map<int, std::vector<MulDesc>> by_variant;
  for (const MulDesc& d : ds) {
    if (d.m <= 0 || d.n <= 0 || d.k <= 0) continue;
    const int v = d.m <= 128 ? 4 : d.m <= 256 ? 3 : d.m <= 512 ? 2 : s.variant;
    const int sk = (int)std::min<int64_t>(kMaxGroup, std::max<int64_t>(1, (d.k + 2047) / 2048));
    if (sk > 1 && d.out == OUT_STORE)
      if ((r = fill_zero(OView{d.C, d.ldc, d.m, words(d.n), tail_of(d.n)}, st)) != GF2_OK) return r;
    if (sk > 1) {
      std::vector<MulDesc> parts;
      plan_splitk(parts, View{d.A, d.lda, d.m, d.k}, View{d.B, d.ldb, d.k, d.n}, d.C, d.ldc, sk);
      by_variant[v].insert(by_variant[v].end(), parts.begin(), parts.end());
    } else {
      by_variant[v].push_back(d);
    }
  }
  for (const auto& kv : by_variant)
    if ((r = m4rm_launch_group(kv.second.data(), (int)kv.second.size(), kv.first, st)) != GF2_OK) return r;
  return GF2_OK;
}

// Strassen leaves in one launch.  Equal tiles run in rounds of one per compute unit; when
// the last round would be less than half full, the leaves whose tiles make up that round
// are cut into k slices (XOR-ed atomically into their zeroed results) that are dispatched
// last, so the short slices spread over the whole machine instead of a few units running
// one more full round.  Example: 32768^3 at two levels, 1408-row tiles: 2352 tiles are
// 9.19 rounds on 256 units; one leaf of 48 tiles becomes 5 x 48 slices of a fifth each.
gf2_status run_leaves(const gf2_schedule& s, const std::vector<MulDesc>& leaves, uint64_t* scratch, hipStream_t st) {
  if (s.kernel != GF2_KERNEL_M4RM || kappa_of(s) < 8 || leaves.size() < 2 || leaves.size() > (size_t)kMaxGroup)
    return run_base(s, leaves, scratch, st);
  const int64_t cus = compute_units();
  std::vector<int64_t> t(leaves.size());
  int64_t T = 0;
  for (size_t i = 0; i < leaves.size(); ++i) T += (t[i] = m4rm_tiles(leaves[i], s.variant));
  const int64_t rounds = (T + cus - 1) / cus, tail = T - (rounds - 1) * cus;
  if (rounds < 2 || 2 * tail > cus) return run_base(s, leaves, scratch, st);
  size_t first = leaves.size();
  int64_t cover = 0;
  while (first > 0 && cover < tail) cover += t[--first];
  const int64_t sk = std::max<int64_t>(2, std::min<int64_t>(8, (cus + cover / 2) / cover));
  std::vector<MulDesc> main(leaves.begin(), leaves.begin() + (std::ptrdiff_t)first), slices, zero;
  for (size_t i = first; i < leaves.size(); ++i) {
    const MulDesc& d = leaves[i];
    const int64_t ski = std::min<int64_t>(sk, words(d.k) / 16);
    if (ski < 2) {
      main.push_back(d);
      continue;
    }
    if (d.out == OUT_STORE) zero.push_back(d);
    plan_splitk(slices, View{d.A, d.lda, d.m, d.k}, View{d.B, d.ldb, d.k, d.n}, d.C, d.ldc, (int)ski);
  }
  if (slices.empty() || main.size() + slices.size() > (size_t)kMaxGroup) return run_base(s, leaves, scratch, st);
  gf2_status r;
  for (const MulDesc& d : zero)
    if ((r = fill_zero(OView{d.C, d.ldc, d.m, words(d.n), tail_of(d.n)}, st)) != GF2_OK) return r;
  main.insert(main.end(), slices.begin(), slices.end());
  return m4rm_launch_group(main.data(), (int)main.size(), s.variant, st, (int)slices.size());
}

// Leaves of the product and the workspace they need: Strassen temporaries first, then
// the base kernel's scratch.  ``base`` == nullptr sizes only.
struct ProductPlan {
  StrassenPlan st;
  std::vector<MulDesc> leaves;   // when not recursing
  std::vector<ExpandOp> expands; // table width < 8: each base product's A as index bytes
  size_t x_words = 0;            // their workspace, after the Strassen temporaries
  size_t scratch_words = 0;      // the base kernel's scratch, after the expansions
  size_t total_words() const { return st.ws_words + x_words + scratch_words; }
};

// Table width < 8: every base product reads an index expansion of its A (m4rm_expand) placed
// in the workspace at ``xbase`` (nullptr: sizing only) and is pointed at it.  Expansions run
// after the Strassen pre-additions, which write some of these A's.
void plan_expansions(ProductPlan& pp, uint64_t* xbase, int kappa, const std::vector<MulDesc*>& ds) {
  for (MulDesc* d : ds) {
    const int64_t ldx = m4rm_expanded_ld(d->k, kappa);
    uint64_t* X = xbase ? xbase + pp.x_words : nullptr;
    pp.x_words += align_words((size_t)((int64_t)d->m * ldx));
    if (xbase) {
      pp.expands.push_back(ExpandOp{d->A, X, d->lda, ldx, d->m, d->k, kappa, 0});
      d->A = X;
      d->lda = ldx;
    }
  }
}

// Two recursion levels with every split exact (padding rule, m a multiple of 4, k and n of 256,
// the node and its children splittable, the grandchildren not): the single-product executor then
// runs both levels' passes fused (strassen_pre2 / strassen_post2), and the node's P0..P6 are not
// needed.  One predicate decides both the plan's workspace and the executor's path.
bool fused_two_levels(int64_t m, int64_t k, int64_t n, const gf2_schedule& s) {
  return s.odd == GF2_ODD_PAD && m % 4 == 0 && k % 256 == 0 && n % 256 == 0 && splittable(m, k, n, s.cutoff) &&
         splittable(m / 2, k / 2, n / 2, s.cutoff) && !splittable(m / 4, k / 4, n / 4, s.cutoff);
}

// ``fusable``: the plan is for the single-product executor, which fuses the passes where
// fused_two_levels holds (batch plans launch every level's passes and keep all buffers).
void plan_product(ProductPlan& pp, uint64_t* base, uint64_t* C, int64_t ldc, const uint64_t* A, int64_t lda,
                  const uint64_t* B, int64_t ldb, int64_t m, int64_t k, int64_t n, bool accumulate,
                  const gf2_schedule& s, bool fusable = false) {
  const int out = accumulate ? OUT_XOR : OUT_STORE;
  const View Av{A, lda, m, k}, Bv{B, ldb, k, n};
  const bool narrow = s.kernel == GF2_KERNEL_M4RM && kappa_of(s) < 8;
  std::vector<MulDesc*> base_ds;
  if (splittable(m, k, n, s.cutoff)) {
    plan_node(pp.st, base, Av, Bv, C, ldc, out, s.cutoff, s.odd, 0, fusable && fused_two_levels(m, k, n, s));
    for (MulDesc& d : pp.st.leaves) base_ds.push_back(&d);
    for (auto& f : pp.st.kfix) base_ds.push_back(&f.second);
    for (MulDesc& d : pp.st.fix) base_ds.push_back(&d);
  } else {
    if (s.splitk > 1 && words(k) > 1) plan_splitk(pp.leaves, Av, Bv, C, ldc, s.splitk);
    else pp.leaves.push_back(make_desc(Av, Bv, C, ldc, out));
    for (MulDesc& d : pp.leaves) base_ds.push_back(&d);
  }
  if (narrow) plan_expansions(pp, base ? base + pp.st.ws_words : nullptr, kappa_of(s), base_ds);
  std::vector<MulDesc> all;
  for (const MulDesc* d : base_ds) all.push_back(*d);
  pp.scratch_words = base_scratch_words(s, all);
}

size_t fast_workspace_words(int64_t m, int64_t k, int64_t n, const gf2_schedule& s) {
  ProductPlan pp;
  plan_product(pp, nullptr, nullptr, words(n), nullptr, words(k), nullptr, words(n), m, k, n, false, s, true);
  return pp.total_words();
}

// Section 4's memory-efficient schedule at the top level (GF2_MEM_LOW): C := A*B with equal
// halves of rows and of (word-aligned) columns, so that each of the seven products fits the
// C quadrant it is written to.
bool two_temp_applies(int64_t m, int64_t k, int64_t n, bool accumulate, const gf2_schedule& s) {
  return s.memory == GF2_MEM_LOW && !accumulate && splittable(m, k, n, s.cutoff) && m % 2 == 0 && n % 128 == 0;
}

struct TwoTemp {
  int64_t m0, k0w, k0, k1, n0w;
  size_t x_words, y_words, sub_words;
  gf2_schedule sub;   // the products below the top level: FAST
};

TwoTemp two_temp_plan(int64_t m, int64_t k, int64_t n, const gf2_schedule& s) {
  TwoTemp t;
  t.m0 = m / 2;
  t.k0w = (words(k) + 1) / 2;
  t.k0 = 64 * t.k0w;
  t.k1 = k - t.k0;
  t.n0w = words(n) / 2;
  t.sub = s;
  t.sub.memory = GF2_MEM_FAST;
  t.x_words = align_words((size_t)(t.m0 * std::max(t.k0w, t.n0w)));
  t.y_words = align_words((size_t)(t.k0 * t.n0w));
  t.sub_words = std::max(fast_workspace_words(t.m0, t.k0, 64 * t.n0w, t.sub),
                         fast_workspace_words(t.m0, t.k1, 64 * t.n0w, t.sub));
  return t;
}

size_t workspace_words(int64_t m, int64_t k, int64_t n, const gf2_schedule& s, bool accumulate = false) {
  if (two_temp_applies(m, k, n, accumulate, s)) {
    const TwoTemp t = two_temp_plan(m, k, n, s);
    return t.x_words + t.y_words + t.sub_words;
  }
  return fast_workspace_words(m, k, n, s);
}

// True when the plan is a node with seven children that are nodes of leaves (two levels), no
// peeling fix-ups, and every split exact: m a multiple of 4, k and n multiples of 256, so that
// every operand of both levels is a 4 x 4 block of equal sub-quadrants.  Plans are built depth
// first, so the pre-additions are [node A, node B, child 0 A, child 0 B, ...] and the
// post-additions [child 0, ..., child 6, node].
bool two_level_exact(const StrassenPlan& pl, int64_t m, int64_t k, int64_t n) {
  if (!pl.kfix.empty() || !pl.fix.empty() || pl.pre.size() != 16 || pl.post.size() != 8 || pl.leaves.size() != 49)
    return false;
  if (m % 4 || k % 256 || n % 256) return false;
  for (size_t i = 0; i < pl.pre.size(); ++i)
    if (pl.pre[i].depth != (i < 2 ? 0 : 1) || pl.pre[i].kind != (int)(i & 1)) return false;
  for (size_t i = 0; i < pl.post.size(); ++i)
    if (pl.post[i].depth != (i < 7 ? 1 : 0)) return false;
  return true;
}

// Launches of one product whose workspace (Strassen temporaries, then the base kernel's
// scratch; ``workspace_words`` of them) starts at ``ws``.  Enqueues kernels only.
gf2_status execute_in(uint64_t* C, int64_t ldc, const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb,
                      int64_t m, int64_t k, int64_t n, bool accumulate, const gf2_schedule& s, hipStream_t st,
                      uint64_t* ws) {
  gf2_status r = GF2_OK;
  ProductPlan pp;
  plan_product(pp, ws, C, ldc, A, lda, B, ldb, m, k, n, accumulate, s, true);
  uint64_t* scratch = ws ? ws + pp.st.ws_words + pp.x_words : nullptr;
  const bool fused = fused_two_levels(m, k, n, s);
  if (fused && !two_level_exact(pp.st, m, k, n))
    return set_error(GF2_ERR_UNSUPPORTED, "internal: a fused two-level plan has an unexpected shape");
  if (fused) {
    // A node and its seven children with every split exact: both levels' pre-additions in one
    // pass, the leaves, both levels' post-additions in one pass.
    const PreOp& ra = pp.st.pre[0];
    const PreOp& rb = pp.st.pre[1];
    Pre2Op pa{}, pb{};
    pa.kind = 0;
    pa.in = ra.in[0].p;
    pa.ldi = ra.in[0].ld;
    pa.R4 = m / 4;
    pa.W4 = words(k) / 4;
    pa.ldn = ra.ldo;
    pb.kind = 1;
    pb.in = rb.in[0].p;
    pb.ldi = rb.in[0].ld;
    pb.R4 = k / 4;
    pb.W4 = words(n) / 4;
    pb.ldn = rb.ldo;
    for (int t = 0; t < 4; ++t) {
      pa.node[t] = ra.out[t];
      pb.node[t] = rb.out[t];
    }
    for (int c = 0; c < 7; ++c) {
      const PreOp& ca = pp.st.pre[2 + 2 * c];
      const PreOp& cb = pp.st.pre[3 + 2 * c];
      for (int t = 0; t < 4; ++t) {
        pa.child[c][t] = ca.out[t];
        pb.child[c][t] = cb.out[t];
      }
      pa.ldc = ca.ldo;
      pb.ldc = cb.ldo;
    }
    if ((r = strassen_pre2(pa, pb, st)) != GF2_OK) return r;
    if ((r = m4rm_expand(pp.expands.data(), (int)pp.expands.size(), st)) != GF2_OK) return r;
    if ((r = run_leaves(s, pp.st.leaves, scratch, st)) != GF2_OK) return r;
    const PostOp& root = pp.st.post[7];
    Post2Op po{};
    po.mode = root.mode;
    for (int c = 0; c < 7; ++c)
      for (int j = 0; j < 7; ++j) po.P[c][j] = pp.st.post[c].P[j];
    po.ldp = pp.st.post[0].ldp;
    po.C = root.c[0].p;
    po.ldc = root.c[0].ld;
    po.R4 = m / 4;
    po.W4 = words(n) / 4;
    return strassen_post2(po, st);
  }
  if (!pp.st.leaves.empty()) {
    // Passes of one recursion depth are independent: pre-additions run depth by depth from
    // the root down, post-additions from the deepest level up, each depth in few launches.
    std::vector<PreOp> pre = pp.st.pre;
    std::vector<PostOp> post = pp.st.post;
    std::stable_sort(pre.begin(), pre.end(), [](const PreOp& a, const PreOp& b) { return a.depth < b.depth; });
    for (size_t i = 0; i < pre.size();) {
      size_t j = i;
      while (j < pre.size() && pre[j].depth == pre[i].depth) ++j;
      if ((r = strassen_pre_ops(pre.data() + i, (int)(j - i), st)) != GF2_OK) return r;
      i = j;
    }
    if ((r = m4rm_expand(pp.expands.data(), (int)pp.expands.size(), st)) != GF2_OK) return r;
    if ((r = run_leaves(s, pp.st.leaves, scratch, st)) != GF2_OK) return r;
    if ((r = run_fixups(s, pp.st.fix, scratch, st)) != GF2_OK) return r;
    int maxd = 0;
    for (const auto& f : pp.st.kfix) maxd = std::max(maxd, f.first);
    for (const PostOp& p : post) maxd = std::max(maxd, p.depth);
    for (int d = maxd; d >= 0; --d) {
      std::vector<PostOp> pd;
      for (const PostOp& p : post)
        if (p.depth == d) pd.push_back(p);
      if ((r = strassen_post_ops(pd.data(), (int)pd.size(), st)) != GF2_OK) return r;
      std::vector<MulDesc> fd;
      for (const auto& f : pp.st.kfix)
        if (f.first == d) fd.push_back(f.second);
      if ((r = run_fixups(s, fd, scratch, st)) != GF2_OK) return r;
    }
    return GF2_OK;
  }
  if (s.splitk > 1 && words(k) > 1 && !accumulate)
    if ((r = fill_zero(OView{C, ldc, m, words(n), tail_of(n)}, st)) != GF2_OK) return r;
  if ((r = m4rm_expand(pp.expands.data(), (int)pp.expands.size(), st)) != GF2_OK) return r;
  return run_base(s, pp.leaves, scratch, st);
}

// The two-temporary schedule (Section 4, memory-efficient form; every addition is XOR):
//   X = S2 = A_NW + A_SW,  Y = T2 = B_SE + B_NE,  C_SW = P6 = X Y
//   X = S0 = A_SW + A_SE,  Y = T0 = B_NE + B_NW,  C_SE = P4 = X Y
//   X = S1 = X + A_NW,     Y = T1 = B_SE + Y,     C_NE = P5 = X Y
//   X = S3 = A_NE + X,     C_NW = P2 = X B_SE,    X = P0 = A_NW B_NW
//   C_NE = U1 = X + C_NE,  C_SW = U2 = C_NE + C_SW,  C_NE = U3 = C_NE + C_SE,
//   C_SE = U6 = C_SW + C_SE,  C_NE = U4 = C_NE + C_NW
//   Y = T3 = Y + B_SW,     C_NW = P3 = A_SE Y,    C_SW = U5 = C_SW + C_NW
//   C_NW = P1 = A_NE B_SW, C_NW = U0 = X + C_NW
// The products run breadth-first below (all their leaves in one launch) in the workspace
// after X and Y, one after another.
gf2_status execute_two_temp(uint64_t* C, int64_t ldc, const uint64_t* A, int64_t lda, const uint64_t* B,
                            int64_t ldb, int64_t m, int64_t k, int64_t n, const gf2_schedule& s, hipStream_t st,
                            uint64_t* ws) {
  const TwoTemp t = two_temp_plan(m, k, n, s);
  const int64_t m0 = t.m0, k0w = t.k0w, k0 = t.k0, k1 = t.k1, n0w = t.n0w, n0 = 64 * n0w;
  uint64_t* X = ws;
  uint64_t* Y = ws + t.x_words;
  uint64_t* sub = Y + t.y_words;
  const uint64_t* A_NW = A;
  const uint64_t* A_NE = A + k0w;
  const uint64_t* A_SW = A + m0 * lda;
  const uint64_t* A_SE = A + m0 * lda + k0w;
  const uint64_t* B_NW = B;
  const uint64_t* B_NE = B + n0w;
  const uint64_t* B_SW = B + k0 * ldb;
  const uint64_t* B_SE = B + k0 * ldb + n0w;
  uint64_t* C_NW = C;
  uint64_t* C_NE = C + n0w;
  uint64_t* C_SW = C + m0 * ldc;
  uint64_t* C_SE = C + m0 * ldc + n0w;
  const uint64_t k1t = tail_of(k1);
  const QView qA_NW{A_NW, lda, m0, k0w, ~0ull}, qA_NE{A_NE, lda, m0, words(k1), k1t};
  const QView qA_SW{A_SW, lda, m0, k0w, ~0ull}, qA_SE{A_SE, lda, m0, words(k1), k1t};
  const QView qB_NW{B_NW, ldb, k0, n0w, ~0ull}, qB_NE{B_NE, ldb, k0, n0w, ~0ull};
  const QView qB_SW{B_SW, ldb, k1, n0w, ~0ull}, qB_SE{B_SE, ldb, k1, n0w, ~0ull};
  const OView oX{X, k0w, m0, k0w, ~0ull}, oY{Y, n0w, k0, n0w, ~0ull};
  const QView qX{X, k0w, m0, k0w, ~0ull}, qY{Y, n0w, k0, n0w, ~0ull}, qP0{X, n0w, m0, n0w, ~0ull};
  const OView oNW{C_NW, ldc, m0, n0w, ~0ull}, oNE{C_NE, ldc, m0, n0w, ~0ull};
  const OView oSW{C_SW, ldc, m0, n0w, ~0ull}, oSE{C_SE, ldc, m0, n0w, ~0ull};
  const QView qNW{C_NW, ldc, m0, n0w, ~0ull}, qNE{C_NE, ldc, m0, n0w, ~0ull};
  const QView qSW{C_SW, ldc, m0, n0w, ~0ull}, qSE{C_SE, ldc, m0, n0w, ~0ull};
  auto prod = [&](uint64_t* c, int64_t lc, const uint64_t* a, int64_t la, const uint64_t* b, int64_t lb, int64_t kk) {
    return execute_in(c, lc, a, la, b, lb, m0, kk, n0, false, t.sub, st, sub);
  };
  gf2_status r;
  if ((r = xor2(oX, qA_NW, qA_SW, GF2_TRACE_PRE, st)) != GF2_OK) return r;     // S2
  if ((r = xor2(oY, qB_SE, qB_NE, GF2_TRACE_PRE, st)) != GF2_OK) return r;     // T2
  if ((r = prod(C_SW, ldc, X, k0w, Y, n0w, k0)) != GF2_OK) return r;           // P6
  if ((r = xor2(oX, qA_SW, qA_SE, GF2_TRACE_PRE, st)) != GF2_OK) return r;     // S0
  if ((r = xor2(oY, qB_NE, qB_NW, GF2_TRACE_PRE, st)) != GF2_OK) return r;     // T0
  if ((r = prod(C_SE, ldc, X, k0w, Y, n0w, k0)) != GF2_OK) return r;           // P4
  if ((r = xor2(oX, qX, qA_NW, GF2_TRACE_PRE, st)) != GF2_OK) return r;        // S1
  if ((r = xor2(oY, qB_SE, qY, GF2_TRACE_PRE, st)) != GF2_OK) return r;        // T1
  if ((r = prod(C_NE, ldc, X, k0w, Y, n0w, k0)) != GF2_OK) return r;           // P5
  if ((r = xor2(oX, qA_NE, qX, GF2_TRACE_PRE, st)) != GF2_OK) return r;        // S3
  if ((r = prod(C_NW, ldc, X, k0w, B_SE, ldb, k1)) != GF2_OK) return r;        // P2
  if ((r = prod(X, n0w, A_NW, lda, B_NW, ldb, k0)) != GF2_OK) return r;        // P0 into X
  if ((r = xor2(oNE, qP0, qNE, GF2_TRACE_POST, st)) != GF2_OK) return r;       // U1
  if ((r = xor2(oSW, qNE, qSW, GF2_TRACE_POST, st)) != GF2_OK) return r;       // U2
  if ((r = xor2(oNE, qNE, qSE, GF2_TRACE_POST, st)) != GF2_OK) return r;       // U3
  if ((r = xor2(oSE, qSW, qSE, GF2_TRACE_POST, st)) != GF2_OK) return r;       // U6
  if ((r = xor2(oNE, qNE, qNW, GF2_TRACE_POST, st)) != GF2_OK) return r;       // U4
  if ((r = xor2(oY, qY, qB_SW, GF2_TRACE_PRE, st)) != GF2_OK) return r;        // T3
  if ((r = prod(C_NW, ldc, A_SE, lda, Y, n0w, k1)) != GF2_OK) return r;        // P3
  if ((r = xor2(oSW, qSW, qNW, GF2_TRACE_POST, st)) != GF2_OK) return r;       // U5
  if ((r = prod(C_NW, ldc, A_NE, lda, B_SW, ldb, k1)) != GF2_OK) return r;     // P1
  return xor2(oNW, qP0, qNW, GF2_TRACE_POST, st);                              // U0
}

// A product in the workspace at ``ws`` (workspace_words of it): two-temporary or breadth-first.
gf2_status execute_ws(uint64_t* C, int64_t ldc, const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb,
                      int64_t m, int64_t k, int64_t n, bool accumulate, const gf2_schedule& s, hipStream_t st,
                      uint64_t* ws) {
  if (two_temp_applies(m, k, n, accumulate, s)) return execute_two_temp(C, ldc, A, lda, B, ldb, m, k, n, s, st, ws);
  return execute_in(C, ldc, A, lda, B, ldb, m, k, n, accumulate, s, st, ws);
}

gf2_status execute(uint64_t* C, int64_t ldc, const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb,
                   int64_t m, int64_t k, int64_t n, bool accumulate, const gf2_schedule& s, hipStream_t st) {
  const size_t need = workspace_words(m, k, n, s, accumulate) * 8;
  WorkspaceLease lease;
  gf2_status r = GF2_OK;
  if (need > 0 && (r = lease.acquire(need, st)) != GF2_OK) return r;
  if (need > 0) lease.used();
  return execute_ws(C, ldc, A, lda, B, ldb, m, k, n, accumulate, s, st, static_cast<uint64_t*>(lease.ptr()));
}

int num_candidates_fwd() { return num_candidates(); }
const gf2_schedule& candidate_fwd(int i) { return candidate(i); }

gf2_status mul_impl(uint64_t* C, int64_t ldc, const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb,
                    int64_t m, int64_t k, int64_t n, bool accumulate, const gf2_schedule* sched, void* stream) {
  g_err[0] = 0;
  gf2_status r = validate(C, ldc, A, lda, B, ldb, m, k, n);
  if (r != GF2_OK) return r;
  if ((r = validate_sched(sched)) != GF2_OK) return r;
  if (m == 0 || n == 0) return GF2_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (k == 0) return accumulate ? GF2_OK : fill_zero(OView{C, ldc, m, words(n), tail_of(n)}, st);
  const gf2_schedule s = resolve(sched, m, k, n, st);
  if ((r = check_resolved(s)) != GF2_OK) return r;
  return execute(C, ldc, A, lda, B, ldb, m, k, n, accumulate, s, st);
}


// ---------------------------------------------------------------- policy and autotuner
std::atomic<int> g_policy{GF2_POLICY_FIXED};
std::atomic<uint64_t> g_policy_epoch{0};   // bumped whenever a policy, model or tune cache changes

struct TuneKey {
  int bm, bk, bn;
  bool operator<(const TuneKey& o) const { return bm != o.bm ? bm < o.bm : bk != o.bk ? bk < o.bk : bn < o.bn; }
};
int tune_bucket(int64_t x) { return (int)std::lround(2.0 * std::log2((double)(x > 0 ? x : 1))); }
std::mutex g_tune_mu;
std::map<TuneKey, std::vector<float>> g_tune;

// The autotuner's operands and stream, shared by every tuning call: one call at a time.
std::recursive_mutex g_tscr_mu;
struct TuneScratch {
  uint64_t* buf = nullptr;
  size_t words = 0;
  hipStream_t stream = nullptr;
  int dev = -1;
} g_tscr;

// ``only`` (optional): time only the candidates whose entry is nonzero (the others stay at -1);
// such a partial result does not enter the autotune cache.
gf2_status autotune_shape(int64_t m, int64_t k, int64_t n, double density, int reps, std::vector<float>& ms,
                          const std::vector<char>* only = nullptr) {
  std::lock_guard<std::recursive_mutex> tlk(g_tscr_mu);
  const int S = num_candidates();
  ms.assign(S, -1.f);
  if (m <= 0 || k <= 0 || n <= 0 || m > INT32_MAX || k > INT32_MAX || n > INT32_MAX)
    return set_error(GF2_ERR_INVALID_ARG, "autotune: dimensions must be in [1, 2^31)");
  if (reps < 1) reps = 1;
  int dev = 0;
  gf2_status r = hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (r != GF2_OK) return r;
  const int64_t Wk = words(k), Wn = words(n);
  const size_t need = (size_t)(m * Wk + k * Wn + m * Wn);
  if (g_tscr.dev != dev) {
    g_tscr = TuneScratch{};
    g_tscr.dev = dev;
  }
  if (!g_tscr.stream && (r = hip_check(hipStreamCreateWithFlags(&g_tscr.stream, hipStreamNonBlocking),
                                       "hipStreamCreate")) != GF2_OK)
    return r;
  if (need > g_tscr.words) {
    if ((r = hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize")) != GF2_OK) return r;
    if (g_tscr.buf) (void)hipFree(g_tscr.buf);
    g_tscr.buf = nullptr;
    g_tscr.words = 0;
    if (hipMalloc(&g_tscr.buf, need * 8) != hipSuccess)
      return set_error(GF2_ERR_ALLOC, "autotune: hipMalloc of %zu bytes failed", need * 8);
    g_tscr.words = need;
  }
  uint64_t* A = g_tscr.buf;
  uint64_t* B = A + m * Wk;
  uint64_t* C = B + k * Wn;
  hipStream_t st = g_tscr.stream;
  if ((r = fill_random(A, m * Wk, 0x1234567ull, density, st)) != GF2_OK) return r;
  if ((r = fill_random(B, k * Wn, 0x7654321ull, density, st)) != GF2_OK) return r;
  hipEvent_t e0, e1;
  if ((r = hip_check(hipEventCreate(&e0), "hipEventCreate")) != GF2_OK) return r;
  if ((r = hip_check(hipEventCreate(&e1), "hipEventCreate")) != GF2_OK) { (void)hipEventDestroy(e0); return r; }
  std::vector<float> t(reps);
  for (int c = 0; c < S; ++c) {
    if (only && !(*only)[c]) continue;
    const gf2_schedule& s = candidate(c);
    if (execute(C, Wn, A, Wk, B, Wn, m, k, n, false, s, st) != GF2_OK) continue;   // warm-up
    bool ok = true;
    for (int i = 0; i < reps && ok; ++i) {
      ok = hipEventRecord(e0, st) == hipSuccess && execute(C, Wn, A, Wk, B, Wn, m, k, n, false, s, st) == GF2_OK &&
           hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
           hipEventElapsedTime(&t[i], e0, e1) == hipSuccess;
    }
    if (!ok) continue;
    std::sort(t.begin(), t.end());
    ms[c] = t[reps / 2];
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  g_err[0] = 0;
  if (!only) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[TuneKey{tune_bucket(m), tune_bucket(k), tune_bucket(n)}] = ms;
    ++g_policy_epoch;
  }
  return hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
}

struct BatchPlanImpl;
gf2_status build_batch_plan(const gf2_problem* probs, int64_t count, BatchPlanImpl& P);
gf2_status autotune_batch_shape(int64_t m, int64_t k, int64_t n, double density, int reps, std::vector<float>& ms,
                                int& copies, const std::vector<char>* only = nullptr);

int argmin_allowed(const std::vector<float>& v, bool batch) {
  int best = -1;
  for (int c = 0; c < (int)v.size(); ++c) {
    if (v[c] < 0 || (batch && !batch_allowed(c))) continue;
    if (best < 0 || v[c] < v[best]) best = c;
  }
  return best;
}

}  // namespace

void bump_policy_epoch() { ++g_policy_epoch; }

int choose_candidate(int64_t m, int64_t k, int64_t n, bool batch, hipStream_t s, bool may_time) {
  const int policy = g_policy.load();
  if (policy == GF2_POLICY_MODEL) {
    const int S = num_candidates();
    std::vector<float> y(2 * S);
    if (model_predict(m, k, n, 0.5, y.data())) {
      const float* yy = y.data() + (batch ? S : 0);   // latency head or batch-throughput head
      int best = -1;
      for (int c = 0; c < S; ++c)
        if ((!batch || batch_allowed(c)) && (best < 0 || yy[c] < yy[best])) best = c;
      if (best >= 0 && batch) {
        const int f = fixed_candidate(m, k, n);
        return model_or_fixed(best, yy[best], f, yy[f]);
      }
      if (best >= 0) return best;
    }
  } else if (policy == GF2_POLICY_AUTOTUNE && m > 0 && k > 0 && n > 0) {
    std::vector<float> ms;
    {
      std::lock_guard<std::mutex> g(g_tune_mu);
      auto it = g_tune.find(TuneKey{tune_bucket(m), tune_bucket(k), tune_bucket(n)});
      if (it != g_tune.end()) ms = it->second;
    }
    if (ms.empty() && may_time) {
      hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
      if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone)
        autotune_shape(m, k, n, 0.5, 3, ms);
    }
    const int best = ms.empty() ? -1 : argmin_allowed(ms, batch);
    if (best >= 0) return best;
  }
  return batch ? fixed_candidate(m, k, n) : -1;
}

gf2_status mul_in_static(uint64_t* C, int64_t ldc, const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb,
                         int64_t m, int64_t k, int64_t n, bool accumulate, const gf2_schedule* sched, void* stream,
                         size_t max_bytes, ScratchFn scratch) {
  g_err[0] = 0;
  gf2_status r = validate(C, ldc, A, lda, B, ldb, m, k, n);
  if (r != GF2_OK) return r;
  if ((r = validate_sched(sched)) != GF2_OK) return r;
  uint64_t* ws = nullptr;
  if ((r = scratch(&ws)) != GF2_OK) return r;
  if (m == 0 || n == 0) return GF2_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (k == 0) return accumulate ? GF2_OK : fill_zero(OView{C, ldc, m, words(n), tail_of(n)}, st);
  const gf2_schedule s = resolve(sched, m, k, n, st, false);
  if ((r = check_resolved(s)) != GF2_OK) return r;
  const size_t need = workspace_words(m, k, n, s, accumulate) * 8;
  if (need > max_bytes)
    return set_error(GF2_ERR_UNSUPPORTED,
                     "%lld x %lld x %lld under schedule (kernel %d, variant %d, cutoff %d, splitk %d) needs %zu bytes "
                     "of workspace; the static scratch holds %zu (choose a schedule with less recursion)",
                     (long long)m, (long long)k, (long long)n, s.kernel, s.variant, s.cutoff, s.splitk, need, max_bytes);
  return execute_ws(C, ldc, A, lda, B, ldb, m, k, n, accumulate, s, st, need > 0 ? ws : nullptr);
}

namespace {

// ---------------------------------------------------------------- batched products

struct BatchPlanImpl {
  uint64_t epoch = 0;                // policy epoch the schedules were chosen under
  std::vector<gf2_problem> probs;
  std::vector<int32_t> sched;
  int device = 0;
  uint64_t* ws = nullptr;            // Strassen temporaries of all products, then base scratch
  MulDesc* d_descs = nullptr;
  BatchItem* d_items = nullptr;
  int* d_counter = nullptr;
  int n_items = 0, grid = 0;
  uint64_t* scratch = nullptr;
  double work = 0;
  std::vector<OView> fills;
  std::vector<PreOp> pre;
  std::vector<PostOp> post;
  std::vector<ExpandOp> expands;     // index expansions of A (table width < 8), after the pre passes
  ExpandOp* d_expands = nullptr;
  int64_t expand_dwords = 0;        // largest expansion, in dwords (launch width)
  // Device copies, pre ops sorted by depth (parents first), post ops deepest first;
  // each group is one multi-op launch.
  OView* d_fills = nullptr;
  PreOp* d_pre = nullptr;
  PostOp* d_post = nullptr;
  struct Group {
    int begin, count;
    int64_t max_elems;
  };
  std::vector<Group> pre_groups, post_groups;
  int64_t fill_max = 0;
  struct Side {
    gf2_schedule s;
    std::vector<MulDesc> ds;
  };
  std::vector<Side> sides;
  hipGraphExec_t exec = nullptr;

  ~BatchPlanImpl() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (ws) (void)hipFree(ws);
    if (d_descs) (void)hipFree(d_descs);
    if (d_items) (void)hipFree(d_items);
    if (d_counter) (void)hipFree(d_counter);
    if (d_fills) (void)hipFree(d_fills);
    if (d_pre) (void)hipFree(d_pre);
    if (d_post) (void)hipFree(d_post);
    if (d_expands) (void)hipFree(d_expands);
  }

  gf2_status enqueue(hipStream_t s) const {
    gf2_status r;
    for (size_t i = 0; i < fills.size(); i += 65535)   // grid y limit
      if ((r = fill_zero_multi(d_fills + i, (int)std::min<size_t>(65535, fills.size() - i), fill_max, s)) != GF2_OK)
        return r;
    for (const Group& gr : pre_groups)
      if ((r = strassen_pre_multi(d_pre + gr.begin, gr.count, gr.max_elems, s)) != GF2_OK) return r;
    if (!expands.empty() && (r = m4rm_expand_list(d_expands, (int)expands.size(), expand_dwords, s)) != GF2_OK)
      return r;
    {
      TraceScope tr(GF2_TRACE_BATCH, n_items, work, s);
      if ((r = m4rm_launch_persistent(d_descs, d_items, n_items, d_counter, grid, s)) != GF2_OK) return r;
    }
    for (const Side& sd : sides)
      if ((r = run_base(sd.s, sd.ds, scratch, s)) != GF2_OK) return r;
    for (const Group& gr : post_groups)
      if ((r = strassen_post_multi(d_post + gr.begin, gr.count, gr.max_elems, s)) != GF2_OK) return r;
    return GF2_OK;
  }
};

struct Interval {
  uintptr_t lo, hi;
};

gf2_status validate_batch(const gf2_problem* probs, int64_t count) {
  if (count < 0) return set_error(GF2_ERR_INVALID_ARG, "negative batch count");
  if (count > 0 && !probs) return set_error(GF2_ERR_INVALID_ARG, "problems array is NULL");
  if (count > (int64_t(1) << 24)) return set_error(GF2_ERR_UNSUPPORTED, "batch larger than 2^24 products");
  std::vector<Interval> cs, ro;
  for (int64_t i = 0; i < count; ++i) {
    const gf2_problem& p = probs[i];
    gf2_status r = validate(p.C, p.ldc, p.A, p.lda, p.B, p.ldb, p.m, p.k, p.n);
    if (r != GF2_OK) return set_error(r, "problem %lld: %s", (long long)i, g_err);
    if (p.schedule < -1 || p.schedule >= num_candidates_fwd())
      return set_error(GF2_ERR_INVALID_ARG, "problem %lld: schedule %d out of range", (long long)i, p.schedule);
    if (p.m == 0 || p.n == 0) continue;
    cs.push_back({(uintptr_t)p.C, (uintptr_t)p.C + (uintptr_t)extent_bytes(p.m, p.ldc, words(p.n))});
    if (p.k > 0) {
      ro.push_back({(uintptr_t)p.A, (uintptr_t)p.A + (uintptr_t)extent_bytes(p.m, p.lda, words(p.k))});
      ro.push_back({(uintptr_t)p.B, (uintptr_t)p.B + (uintptr_t)extent_bytes(p.k, p.ldb, words(p.n))});
    }
  }
  auto by_lo = [](const Interval& x, const Interval& y) { return x.lo < y.lo; };
  std::sort(cs.begin(), cs.end(), by_lo);
  for (size_t i = 1; i < cs.size(); ++i)
    if (cs[i].lo < cs[i - 1].hi) return set_error(GF2_ERR_ALIAS, "two outputs of the batch overlap");
  // Union of the read-only ranges, then each output against it.
  std::sort(ro.begin(), ro.end(), by_lo);
  std::vector<Interval> uni;
  for (const Interval& x : ro) {
    if (!uni.empty() && x.lo <= uni.back().hi) uni.back().hi = std::max(uni.back().hi, x.hi);
    else uni.push_back(x);
  }
  for (const Interval& c : cs) {
    auto it = std::upper_bound(uni.begin(), uni.end(), c, by_lo);   // first range starting after c.lo
    if (it != uni.end() && it->lo < c.hi) return set_error(GF2_ERR_ALIAS, "an output overlaps an input of the batch");
    if (it != uni.begin() && std::prev(it)->hi > c.lo)
      return set_error(GF2_ERR_ALIAS, "an output overlaps an input of the batch");
  }
  return GF2_OK;
}

// Relative run time of one tile, for the queue order: phases x (rows + the table build).
double tile_cost(const MulDesc& d, int variant, int kappa, int tm) {
  const int64_t bm = m4rm_tile_rows(variant), pr = m4rm_phase_rows(variant, kappa);
  const int64_t rows = std::min<int64_t>(bm, d.m - (int64_t)tm * bm);
  return (double)((d.k + pr - 1) / pr) * (double)(rows * (pr / kappa) / 2 + (1 << kappa));
}

gf2_status build_batch_plan(const gf2_problem* probs, int64_t count, BatchPlanImpl& P) {
  gf2_status r = validate_batch(probs, count);
  if (r != GF2_OK) return r;
  if ((r = hip_check(hipGetDevice(&P.device), "hipGetDevice")) != GF2_OK) return r;
  P.epoch = g_policy_epoch.load();
  P.probs.assign(probs, probs + count);
  P.sched.resize(count);
  // Pass 1: schedules and workspace sizes.
  std::vector<size_t> ws_off(count + 1, 0);
  size_t scratch_words = 0;
  std::vector<int> model_pick;
  if (g_policy.load() == GF2_POLICY_MODEL && model_available()) {
    std::vector<float> feats;
    std::vector<int> fixed;
    for (int64_t i = 0; i < count; ++i)
      if (probs[i].schedule < 0) {
        feats.insert(feats.end(), {(float)std::log2((double)std::max<int64_t>(probs[i].m, 1)),
                                   (float)std::log2((double)std::max<int64_t>(probs[i].k, 1)),
                                   (float)std::log2((double)std::max<int64_t>(probs[i].n, 1)), 0.5f});
        fixed.push_back(fixed_candidate(probs[i].m, probs[i].k, probs[i].n));
      }
    std::vector<uint8_t> allowed(num_candidates());
    for (int c = 0; c < num_candidates(); ++c) allowed[c] = batch_allowed(c) ? 1 : 0;
    if ((r = model_choose_batch(feats, allowed.data(), fixed, model_pick)) != GF2_OK) return r;
  }
  size_t pick = 0, mfma_scratch = 0;
  for (int64_t i = 0; i < count; ++i) {
    const gf2_problem& p = probs[i];
    if (p.schedule >= 0) P.sched[i] = p.schedule;
    else if (!model_pick.empty() && model_pick[pick] >= 0) P.sched[i] = model_pick[pick++];
    else P.sched[i] = choose_candidate(p.m, p.k, p.n, true, nullptr);
    size_t w = 0;
    if (p.m > 0 && p.n > 0 && p.k > 0) {
      ProductPlan pp;
      plan_product(pp, nullptr, p.C, p.ldc, p.A, p.lda, p.B, p.ldb, p.m, p.k, p.n, p.accumulate != 0,
                   candidate_fwd(P.sched[i]));
      w = pp.st.ws_words + pp.x_words;
      // Products on the int8 matrix core share one grouped launch, so their transposed Bs
      // coexist (sum); other base cases reuse the scratch one product at a time (max).
      if (candidate_fwd(P.sched[i]).kernel == GF2_KERNEL_MFMA) mfma_scratch += pp.scratch_words;
      else scratch_words = std::max(scratch_words, pp.scratch_words);
    }
    ws_off[i + 1] = ws_off[i] + w;
  }
  scratch_words = std::max(scratch_words, mfma_scratch);
  const size_t total = ws_off[count] + scratch_words;
  if (total > 0) {
    if (fault_alloc()) return set_error(GF2_ERR_ALLOC, "injected allocation failure (GF2_FAULT_ALLOC)");
    if (hipMalloc(&P.ws, total * 8) != hipSuccess) {
      P.ws = nullptr;
      return set_error(GF2_ERR_ALLOC, "hipMalloc of %zu bytes of batch workspace failed", total * 8);
    }
  }
  P.scratch = P.ws ? P.ws + ws_off[count] : nullptr;
  // Pass 2: descriptors, queue items, side launches, fills, Strassen passes.
  std::vector<MulDesc> descs;
  std::vector<BatchItem> items;
  std::vector<double> cost;
  auto route = [&](const gf2_schedule& s, const std::vector<MulDesc>& leaves) {
    const int kappa = kappa_of(s);
    if (s.kernel == GF2_KERNEL_M4RM && m4rm_batchable(s.variant)) {
      for (const MulDesc& d : leaves) {
        const int di = (int)descs.size();
        descs.push_back(d);
        const int64_t bm = m4rm_tile_rows(s.variant), tw = m4rm_tile_words(s.variant);
        const int64_t tms = (d.m + bm - 1) / bm, tns = (words(d.n) + tw - 1) / tw;
        P.work += (double)d.m * ((d.k + kappa - 1) / kappa) * (double)words(d.n);
        for (int64_t tm = 0; tm < tms; ++tm)
          for (int64_t tn = 0; tn < tns; ++tn) {
            items.push_back(BatchItem{di, (int32_t)tm, (int32_t)tn, s.variant | (kappa << 8)});
            cost.push_back(tile_cost(d, s.variant, kappa, (int)tm));
          }
      }
      return;
    }
    for (auto& sd : P.sides)
      if (sd.s.kernel == s.kernel && sd.s.variant == s.variant && kappa_of(sd.s) == kappa) {
        sd.ds.insert(sd.ds.end(), leaves.begin(), leaves.end());
        return;
      }
    P.sides.push_back({s, leaves});
  };
  for (int64_t i = 0; i < count; ++i) {
    const gf2_problem& p = probs[i];
    if (p.m == 0 || p.n == 0) continue;
    const gf2_schedule& s = candidate_fwd(P.sched[i]);
    if (p.k == 0) {
      if (!p.accumulate) P.fills.push_back(OView{p.C, p.ldc, p.m, words(p.n), tail_of(p.n)});
      continue;
    }
    ProductPlan pp;
    plan_product(pp, P.ws ? P.ws + ws_off[i] : nullptr, p.C, p.ldc, p.A, p.lda, p.B, p.ldb, p.m, p.k, p.n,
                 p.accumulate != 0, s);
    if (!pp.st.kfix.empty() || !pp.st.fix.empty())
      return set_error(GF2_ERR_UNSUPPORTED, "peeling is not supported in batches");
    P.expands.insert(P.expands.end(), pp.expands.begin(), pp.expands.end());
    if (!pp.st.leaves.empty()) {
      P.pre.insert(P.pre.end(), pp.st.pre.begin(), pp.st.pre.end());
      P.post.insert(P.post.end(), pp.st.post.begin(), pp.st.post.end());
      route(s, pp.st.leaves);
    } else {
      if (s.splitk > 1 && words(p.k) > 1 && !p.accumulate)
        P.fills.push_back(OView{p.C, p.ldc, p.m, words(p.n), tail_of(p.n)});
      route(s, pp.leaves);
    }
  }
  // Longest tiles first, so the queue ends with short work.
  std::vector<size_t> order(items.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return cost[x] > cost[y]; });
  std::vector<BatchItem> sorted(items.size());
  for (size_t i = 0; i < order.size(); ++i) sorted[i] = items[order[i]];
  if (sorted.size() > (size_t)INT32_MAX) return set_error(GF2_ERR_UNSUPPORTED, "too many tiles in one batch");
  P.n_items = (int)sorted.size();
  int cus = 0;
  if ((r = hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, P.device),
                     "hipDeviceGetAttribute")) != GF2_OK)
    return r;
  P.grid = std::max(1, std::min(cus, P.n_items));
  auto upload = [&](void** dst, const void* src, size_t bytes) -> gf2_status {
    if (hipMalloc(dst, bytes ? bytes : 8) != hipSuccess) {
      *dst = nullptr;
      return set_error(GF2_ERR_ALLOC, "hipMalloc of %zu bytes for batch descriptors failed", bytes);
    }
    return bytes ? hip_check(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice), "hipMemcpy") : GF2_OK;
  };
  if ((r = upload((void**)&P.d_descs, descs.data(), descs.size() * sizeof(MulDesc))) != GF2_OK) return r;
  if ((r = upload((void**)&P.d_items, sorted.data(), sorted.size() * sizeof(BatchItem))) != GF2_OK) return r;
  if ((r = upload((void**)&P.d_counter, nullptr, 0)) != GF2_OK) return r;
  // Auxiliary passes: fills in one launch, Strassen passes in one launch per depth.
  for (const OView& o : P.fills) P.fill_max = std::max(P.fill_max, o.rows * o.wds);
  std::stable_sort(P.pre.begin(), P.pre.end(), [](const PreOp& x, const PreOp& y) { return x.depth < y.depth; });
  std::stable_sort(P.post.begin(), P.post.end(), [](const PostOp& x, const PostOp& y) { return x.depth > y.depth; });
  auto groups = [](const auto& ops, std::vector<BatchPlanImpl::Group>& out, auto elems) {
    for (int i = 0; i < (int)ops.size();) {
      int j = i;
      int64_t mx = 0;
      while (j < (int)ops.size() && ops[j].depth == ops[i].depth && j - i < 65535) mx = std::max(mx, elems(ops[j++]));
      out.push_back({i, j - i, mx});
      i = j;
    }
  };
  groups(P.pre, P.pre_groups, [](const PreOp& o) { return o.R * o.Wd; });
  groups(P.post, P.post_groups, [](const PostOp& o) { return o.c[0].rows * o.c[0].wds; });
  if ((r = upload((void**)&P.d_fills, P.fills.data(), P.fills.size() * sizeof(OView))) != GF2_OK) return r;
  if ((r = upload((void**)&P.d_pre, P.pre.data(), P.pre.size() * sizeof(PreOp))) != GF2_OK) return r;
  if ((r = upload((void**)&P.d_post, P.post.data(), P.post.size() * sizeof(PostOp))) != GF2_OK) return r;
  for (const ExpandOp& o : P.expands) P.expand_dwords = std::max<int64_t>(P.expand_dwords, (int64_t)o.m * 2 * o.ldx);
  if ((r = upload((void**)&P.d_expands, P.expands.data(), P.expands.size() * sizeof(ExpandOp))) != GF2_OK) return r;
  return GF2_OK;
}

// Graph capture of a plan's launches on a private stream.
gf2_status capture_plan(BatchPlanImpl& P) {
  hipStream_t cs = nullptr;
  gf2_status r = hip_check(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate");
  if (r != GF2_OK) return r;
  hipGraph_t graph = nullptr;
  trace_suspend(true);
  r = hip_check(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  if (r == GF2_OK) {
    gf2_status er = P.enqueue(cs);
    gf2_status ec = hip_check(hipStreamEndCapture(cs, &graph), "hipStreamEndCapture");
    r = er != GF2_OK ? er : ec;
  }
  trace_suspend(false);
  if (r == GF2_OK) r = hip_check(hipGraphInstantiate(&P.exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
  if (graph) (void)hipGraphDestroy(graph);
  (void)hipStreamDestroy(cs);
  return r;
}

std::mutex g_batch_mu;
std::vector<std::unique_ptr<BatchPlanImpl>> g_batch_cache;
constexpr size_t kBatchCacheMax = 8;


// Per-product time of every candidate inside a batch of R copies of the product.
gf2_status autotune_batch_shape(int64_t m, int64_t k, int64_t n, double density, int reps, std::vector<float>& ms,
                                int& copies, const std::vector<char>* only) {
  std::lock_guard<std::recursive_mutex> tlk(g_tscr_mu);
  const int S = num_candidates();
  ms.assign(S, -1.f);
  if (m <= 0 || k <= 0 || n <= 0 || m > INT32_MAX || k > INT32_MAX || n > INT32_MAX)
    return set_error(GF2_ERR_INVALID_ARG, "autotune: dimensions must be in [1, 2^31)");
  if (reps < 1) reps = 1;
  // Enough copies that even the tallest persistent tile (1024 rows x 16 words) gives ~2048
  // tiles, i.e. the batch fills every compute unit several times over, as in a real batch.
  // Every copy has its own A, B and C (at most 512 MiB in all): with shared operands the
  // re-reads of A and B by a product's tiles would hit in cache across copies, which favours
  // the tiles that re-read operands most (the narrow ones) over what a real batch sees.
  const int64_t Wk = words(k), Wn = words(n);
  const double vol = (double)m * (double)k * (double)n;
  const int64_t tiles1024 = ((m + 1023) / 1024) * ((Wn + 15) / 16);
  const int64_t per_copy = m * Wk + k * Wn + m * Wn;   // words
  int64_t R = std::max<int64_t>((2048 + tiles1024 - 1) / tiles1024, (int64_t)std::llround(8e8 / vol));
  R = std::max<int64_t>(2, std::min<int64_t>(R, 512));
  R = std::max<int64_t>(1, std::min<int64_t>(R, (int64_t)((512ll << 20) / (8 * per_copy))));
  copies = (int)R;
  int dev = 0;
  gf2_status r = hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (r != GF2_OK) return r;
  const size_t need = (size_t)(R * per_copy);
  if (g_tscr.dev != dev) {
    g_tscr = TuneScratch{};
    g_tscr.dev = dev;
  }
  if (!g_tscr.stream && (r = hip_check(hipStreamCreateWithFlags(&g_tscr.stream, hipStreamNonBlocking),
                                       "hipStreamCreate")) != GF2_OK)
    return r;
  if (need > g_tscr.words) {
    if ((r = hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize")) != GF2_OK) return r;
    if (g_tscr.buf) (void)hipFree(g_tscr.buf);
    g_tscr.buf = nullptr;
    g_tscr.words = 0;
    if (hipMalloc(&g_tscr.buf, need * 8) != hipSuccess)
      return set_error(GF2_ERR_ALLOC, "autotune: hipMalloc of %zu bytes failed", need * 8);
    g_tscr.words = need;
  }
  uint64_t* A = g_tscr.buf;                 // R copies of A, then of B, then of C
  uint64_t* B = A + R * m * Wk;
  uint64_t* C = B + R * k * Wn;
  hipStream_t st = g_tscr.stream;
  if ((r = fill_random(A, R * m * Wk, 0x1234567ull, density, st)) != GF2_OK) return r;
  if ((r = fill_random(B, R * k * Wn, 0x7654321ull, density, st)) != GF2_OK) return r;
  std::vector<gf2_problem> probs(R);
  hipEvent_t e0, e1;
  if ((r = hip_check(hipEventCreate(&e0), "hipEventCreate")) != GF2_OK) return r;
  if ((r = hip_check(hipEventCreate(&e1), "hipEventCreate")) != GF2_OK) { (void)hipEventDestroy(e0); return r; }
  std::vector<float> t(reps);
  for (int c = 0; c < S; ++c) {
    if (only && !(*only)[c]) continue;
    for (int64_t i = 0; i < R; ++i)
      probs[i] = gf2_problem{A + i * m * Wk, B + i * k * Wn, C + i * m * Wn, m, k, n, Wk, Wn, Wn, 0, c};
    BatchPlanImpl P;
    if (build_batch_plan(probs.data(), R, P) != GF2_OK || P.enqueue(st) != GF2_OK) continue;
    bool ok = true;
    for (int i = 0; i < reps && ok; ++i) {
      ok = hipEventRecord(e0, st) == hipSuccess && P.enqueue(st) == GF2_OK && hipEventRecord(e1, st) == hipSuccess &&
           hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&t[i], e0, e1) == hipSuccess;
    }
    if (hipStreamSynchronize(st) != hipSuccess) ok = false;
    if (!ok) continue;
    std::sort(t.begin(), t.end());
    ms[c] = t[reps / 2] / (float)R;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  g_err[0] = 0;
  return hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
}

bool same_batch(const BatchPlanImpl& P, const gf2_problem* probs, int64_t count, int device) {
  return P.device == device && P.epoch == g_policy_epoch.load() && (int64_t)P.probs.size() == count &&
         std::memcmp(P.probs.data(), probs, sizeof(gf2_problem) * (size_t)count) == 0;
}

}  // namespace
}  // namespace gf2

using namespace gf2;

extern "C" {

gf2_status gf2_mul(uint64_t* C, int64_t ldc, const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb,
                   int64_t m, int64_t k, int64_t n, void* stream) {
  return mul_impl(C, ldc, A, lda, B, ldb, m, k, n, false, nullptr, stream);
}

gf2_status gf2_addmul(uint64_t* C, int64_t ldc, const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb,
                      int64_t m, int64_t k, int64_t n, void* stream) {
  return mul_impl(C, ldc, A, lda, B, ldb, m, k, n, true, nullptr, stream);
}

gf2_status gf2_mul_sched(uint64_t* C, int64_t ldc, const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb,
                         int64_t m, int64_t k, int64_t n, int32_t accumulate, const gf2_schedule* sched,
                         void* stream) {
  return mul_impl(C, ldc, A, lda, B, ldb, m, k, n, accumulate != 0, sched, stream);
}

gf2_status gf2_mul_batched(const gf2_problem* probs, int64_t count, void* stream) {
  g_err[0] = 0;
  if (count == 0) return GF2_OK;
  gf2_status r = validate_batch(probs, count);
  if (r != GF2_OK) return r;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int dev = 0;
  if ((r = hip_check(hipGetDevice(&dev), "hipGetDevice")) != GF2_OK) return r;
  std::lock_guard<std::mutex> lk(g_batch_mu);
  BatchPlanImpl* plan = nullptr;
  if (probs)
    for (auto& p : g_batch_cache)
      if (same_batch(*p, probs, count, dev)) { plan = p.get(); break; }
  if (!plan) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if ((r = hip_check(hipStreamIsCapturing(st, &cs), "hipStreamIsCapturing")) != GF2_OK) return r;
    if (cs != hipStreamCaptureStatusNone)
      return set_error(GF2_ERR_CAPTURE, "a new batch cannot be planned under stream capture; use gf2_batch_plan_*");
    auto P = std::make_unique<BatchPlanImpl>();
    if ((r = build_batch_plan(probs, count, *P)) != GF2_OK) return r;
    if ((r = capture_plan(*P)) != GF2_OK) return r;
    if (g_batch_cache.size() >= kBatchCacheMax) {
      if ((r = hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize")) != GF2_OK) return r;
      g_batch_cache.clear();
    }
    g_batch_cache.push_back(std::move(P));
    plan = g_batch_cache.back().get();
  }
  TraceScope tr(GF2_TRACE_BATCH, plan->n_items, plan->work, st);
  return hip_check(hipGraphLaunch(plan->exec, st), "hipGraphLaunch");
}

struct gf2_batch_plan_s {
  BatchPlanImpl impl;
};

gf2_status gf2_batch_plan_create(const gf2_problem* probs, int64_t count, gf2_batch_plan* out) {
  g_err[0] = 0;
  if (!out) return set_error(GF2_ERR_INVALID_ARG, "output plan pointer is NULL");
  *out = nullptr;
  auto p = std::make_unique<gf2_batch_plan_s>();
  gf2_status r = build_batch_plan(probs, count, p->impl);
  if (r != GF2_OK) return r;
  *out = p.release();
  return GF2_OK;
}

gf2_status gf2_batch_plan_execute(gf2_batch_plan plan, void* stream) {
  g_err[0] = 0;
  if (!plan) return set_error(GF2_ERR_INVALID_ARG, "plan is NULL");
  return plan->impl.enqueue(static_cast<hipStream_t>(stream));
}

gf2_status gf2_batch_plan_destroy(gf2_batch_plan plan) {
  if (!plan) return GF2_OK;
  gf2_status r = hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
  delete plan;
  return r;
}

int32_t gf2_batch_plan_schedule(gf2_batch_plan plan, int64_t i) {
  if (!plan || i < 0 || i >= (int64_t)plan->impl.sched.size()) return -1;
  return plan->impl.sched[i];
}

gf2_status gf2_set_policy(int32_t policy) {
  if (policy < GF2_POLICY_FIXED || policy > GF2_POLICY_MODEL)
    return set_error(GF2_ERR_INVALID_ARG, "unknown policy %d", policy);
  g_policy.store(policy);
  ++g_policy_epoch;
  return GF2_OK;
}

int32_t gf2_get_policy(void) { return g_policy.load(); }

gf2_status gf2_resolve_schedule(int64_t m, int64_t k, int64_t n, const gf2_schedule* req, gf2_schedule* out) {
  g_err[0] = 0;
  if (m < 0 || k < 0 || n < 0) return set_error(GF2_ERR_INVALID_ARG, "negative dimension");
  if (!out) return set_error(GF2_ERR_INVALID_ARG, "out is NULL");
  gf2_status r = validate_sched(req);
  if (r != GF2_OK) return r;
  *out = resolve(req, m, k, n, nullptr);
  return GF2_OK;
}

int32_t gf2_choose_schedule(int64_t m, int64_t k, int64_t n, int32_t batch) {
  if (m < 0 || k < 0 || n < 0) return -1;
  const int c = choose_candidate(m, k, n, batch != 0, nullptr);
  return c >= 0 ? c : fixed_candidate(m, k, n);
}

gf2_status gf2_autotune(int64_t m, int64_t k, int64_t n, double density, int32_t reps, float* ms, int32_t* best) {
  g_err[0] = 0;
  if (density < 0 || density > 1) return set_error(GF2_ERR_INVALID_ARG, "density must be in [0, 1]");
  std::vector<float> v;
  gf2_status r = autotune_shape(m, k, n, density, reps, v);
  if (r != GF2_OK) return r;
  if (ms) std::copy(v.begin(), v.end(), ms);
  if (best) *best = argmin_allowed(v, false);
  return GF2_OK;
}

gf2_status gf2_autotune_batch(int64_t m, int64_t k, int64_t n, double density, int32_t reps, float* ms,
                              int32_t* best, int32_t* copies) {
  g_err[0] = 0;
  if (density < 0 || density > 1) return set_error(GF2_ERR_INVALID_ARG, "density must be in [0, 1]");
  std::vector<float> v;
  int R = 0;
  gf2_status r = autotune_batch_shape(m, k, n, density, reps, v, R);
  if (r != GF2_OK) return r;
  if (ms) std::copy(v.begin(), v.end(), ms);
  if (best) *best = argmin_allowed(v, true);
  if (copies) *copies = R;
  return GF2_OK;
}

gf2_status gf2_autotune_candidates(int64_t m, int64_t k, int64_t n, double density, int32_t reps, int32_t batch,
                                   const int32_t* candidates, int32_t count, float* ms, int32_t* copies) {
  g_err[0] = 0;
  if (density < 0 || density > 1) return set_error(GF2_ERR_INVALID_ARG, "density must be in [0, 1]");
  const int S = num_candidates();
  if (count < 0 || (count > 0 && !candidates)) return set_error(GF2_ERR_INVALID_ARG, "candidate list is invalid");
  std::vector<char> only(S, 0);
  for (int32_t i = 0; i < count; ++i) {
    if (candidates[i] < 0 || candidates[i] >= S)
      return set_error(GF2_ERR_INVALID_ARG, "candidate index %d out of range [0, %d)", candidates[i], S);
    only[candidates[i]] = 1;
  }
  std::vector<float> v;
  int R = 1;
  const gf2_status r = batch ? autotune_batch_shape(m, k, n, density, reps, v, R, &only)
                             : autotune_shape(m, k, n, density, reps, v, &only);
  if (r != GF2_OK) return r;
  if (ms) std::copy(v.begin(), v.end(), ms);
  if (copies) *copies = R;
  return GF2_OK;
}

gf2_status gf2_autotune_save(const char* path) {
  if (!path) return set_error(GF2_ERR_INVALID_ARG, "path is NULL");
  std::ofstream f(path);
  if (!f) return set_error(GF2_ERR_INVALID_ARG, "cannot write %s", path);
  std::lock_guard<std::mutex> g(g_tune_mu);
  for (const auto& kv : g_tune) {
    f << kv.first.bm << ' ' << kv.first.bk << ' ' << kv.first.bn;
    for (float x : kv.second) f << ' ' << x;
    f << '\n';
  }
  return f ? GF2_OK : set_error(GF2_ERR_INVALID_ARG, "write to %s failed", path);
}

gf2_status gf2_autotune_load(const char* path) {
  if (!path) return set_error(GF2_ERR_INVALID_ARG, "path is NULL");
  std::ifstream f(path);
  if (!f) return set_error(GF2_ERR_INVALID_ARG, "cannot read %s", path);
  std::map<TuneKey, std::vector<float>> loaded;
  TuneKey key;
  const int S = num_candidates();
  while (f >> key.bm >> key.bk >> key.bn) {
    std::vector<float> v(S);
    for (int c = 0; c < S; ++c)
      if (!(f >> v[c])) return set_error(GF2_ERR_INVALID_ARG, "%s: truncated entry (cache left unchanged)", path);
    loaded[key] = v;
  }
  if (!f.eof()) return set_error(GF2_ERR_INVALID_ARG, "%s: malformed (cache left unchanged)", path);
  std::lock_guard<std::mutex> g(g_tune_mu);
  for (auto& kv : loaded) g_tune[kv.first] = kv.second;
  ++g_policy_epoch;
  return GF2_OK;
}

void gf2_autotune_clear(void) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune.clear();
  ++g_policy_epoch;
}

int32_t gf2_kernel_variants(int32_t kernel) {
  switch (kernel) {
    case GF2_KERNEL_M4RM: return m4rm_num_variants();
    case GF2_KERNEL_MFMA: return 1;
    case GF2_KERNEL_CUBIC: return 1;
    default: return 0;
  }
}

size_t gf2_workspace_bytes(int64_t m, int64_t k, int64_t n, const gf2_schedule* sched) {
  if (m <= 0 || k <= 0 || n <= 0) return 0;
  const gf2_schedule s = resolve(sched, m, k, n, nullptr);
  return workspace_words(m, k, n, s) * 8;
}

gf2_status gf2_reserve_workspace(size_t bytes) {
  g_err[0] = 0;
  WorkspaceLease lease;
  gf2_status r = lease.acquire(bytes, nullptr);
  if (r != GF2_OK) return r;
  return hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
}

const char* gf2_status_string(gf2_status s) {
  switch (s) {
    case GF2_OK: return "GF2_OK";
    case GF2_ERR_INVALID_ARG: return "GF2_ERR_INVALID_ARG";
    case GF2_ERR_ALIAS: return "GF2_ERR_ALIAS";
    case GF2_ERR_ALLOC: return "GF2_ERR_ALLOC";
    case GF2_ERR_CAPTURE: return "GF2_ERR_CAPTURE";
    case GF2_ERR_DEVICE: return "GF2_ERR_DEVICE";
    case GF2_ERR_UNSUPPORTED: return "GF2_ERR_UNSUPPORTED";
  }
  return "GF2_ERR_UNKNOWN";
}

const char* gf2_last_error(void) { return g_err; }

void gf2_shutdown(void) {
  gf2_set_model(nullptr, 0, nullptr);
  {
    std::lock_guard<std::recursive_mutex> tlk(g_tscr_mu);
    if (g_tscr.buf) (void)hipFree(g_tscr.buf);
    if (g_tscr.stream) (void)hipStreamDestroy(g_tscr.stream);
    g_tscr = TuneScratch{};
  }
  {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    if (!g_batch_cache.empty()) (void)hipDeviceSynchronize();
    g_batch_cache.clear();
  }
  for (auto& d : g_dev) {
    std::lock_guard<std::mutex> g(d.mu);
    if (d.base || !d.retired.empty()) (void)hipDeviceSynchronize();
    if (d.base) (void)hipFree(d.base);
    for (void* p : d.retired) (void)hipFree(p);
    if (d.last) (void)hipEventDestroy(d.last);
    d.base = nullptr;
    d.bytes = 0;
    d.last = nullptr;
    d.has_last = false;
    d.captured = false;
    d.retired.clear();
  }
}

}  // extern "C"
