// C-ABI entry points: argument validation, schedule resolution, workspace, and the
// Strassen-Winograd executor (Section 4, Algorithm 4) over the base-case kernels.
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
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
    if (need > ds_->bytes) {
      hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
      st = hip_check(hipStreamIsCapturing(s, &cs), "hipStreamIsCapturing");
      if (st != GF2_OK) return st;
      if (cs != hipStreamCaptureStatusNone)
        return set_error(GF2_ERR_CAPTURE, "needs %zu bytes of workspace under stream capture; call "
                         "gf2_reserve_workspace first", need);
      if (fault_alloc()) return set_error(GF2_ERR_ALLOC, "injected allocation failure (GF2_FAULT_ALLOC)");
      st = hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
      if (st != GF2_OK) return st;
      if (ds_->base) (void)hipFree(ds_->base);
      ds_->base = nullptr;
      ds_->bytes = 0;
      const size_t grow = need + need / 4 + (1u << 20);
      if (hipMalloc(&ds_->base, grow) != hipSuccess) {
        ds_->base = nullptr;
        return set_error(GF2_ERR_ALLOC, "hipMalloc of %zu bytes of workspace failed", grow);
      }
      ds_->bytes = grow;
    }
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

// Default schedule for a shape (the fixed heuristic, used when nothing better is known):
// the tallest M4RM tile that still gives every compute unit work, two Strassen-Winograd
// levels once the smallest dimension reaches 8192, and k split when there are too few
// C tiles to fill 256 compute units.
int64_t tiles_for(int64_t m, int64_t n, int v) {
  const int64_t bm = m4rm_tile_rows(v), tw = m4rm_tile_words(v);
  return ((m + bm - 1) / bm) * ((words(n) + tw - 1) / tw);
}

gf2_schedule default_schedule(int64_t m, int64_t k, int64_t n) {
  gf2_schedule s{};
  s.kernel = GF2_KERNEL_M4RM;
  const int64_t mn = m < n ? (m < k ? m : k) : (n < k ? n : k);
  s.cutoff = mn >= 8192 ? (int32_t)(mn / 4) : 0;
  const int64_t lm = s.cutoff ? (m + 3) / 4 : m, ln = s.cutoff ? (n + 3) / 4 : n;
  const int64_t leaves = s.cutoff ? 49 : 1;
  const int order[] = {0, 1, 2, 3};
  int v = 3;
  for (int vi : order) {
    if (tiles_for(lm, ln, vi) * leaves >= 512) { v = vi; break; }
  }
  s.variant = v;
  const int64_t tiles = tiles_for(lm, ln, v) * leaves;
  int sk = 1;
  if (!s.cutoff)
    while (tiles * sk < 512 && k / (64 * (sk * 2)) >= 16 && sk * 2 <= kMaxGroup) sk *= 2;
  s.splitk = sk;
  return s;
}

gf2_schedule resolve(const gf2_schedule* req, int64_t m, int64_t k, int64_t n) {
  gf2_schedule s = default_schedule(m, k, n);
  {
    std::lock_guard<std::mutex> g(g_sched_mu);
    if (!req && g_has_override) req = &g_override;
  }
  if (req) {
    if (req->kernel != GF2_KERNEL_AUTO) s.kernel = req->kernel;
    if (req->kernel != GF2_KERNEL_AUTO || req->variant) s.variant = req->variant;
    s.cutoff = req->cutoff;
    if (req->splitk > 0) s.splitk = req->splitk;
  }
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
  if (s.kernel == GF2_KERNEL_CUBIC)
    for (const MulDesc& d : ds) w = std::max(w, cubic_scratch_words(d));
  return w;
}

// Base-case products launched together.
gf2_status run_base(const gf2_schedule& s, const std::vector<MulDesc>& ds, uint64_t* scratch, hipStream_t st) {
  if (ds.empty()) return GF2_OK;
  switch (s.kernel) {
    case GF2_KERNEL_MFMA:
      return mfma_launch_group(ds.data(), (int)ds.size(), st);
    case GF2_KERNEL_CUBIC:
      for (const MulDesc& d : ds) {
        gf2_status r = cubic_launch(d, scratch, st);
        if (r != GF2_OK) return r;
      }
      return GF2_OK;
    case GF2_KERNEL_M4RM:
    default:
      return m4rm_launch_group(ds.data(), (int)ds.size(), s.variant, st);
  }
}

struct PreOp { int kind; QView in[4]; uint64_t* out[4]; int64_t ldo, R, Wd; };
struct PostOp { const uint64_t* P[7]; int64_t ldp; OView c[4]; int mode; };

struct StrassenPlan {
  std::vector<PreOp> pre;
  std::vector<MulDesc> leaves;
  std::vector<PostOp> post;
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
void plan_node(StrassenPlan& pl, uint64_t* base, const View& A, const View& B, uint64_t* C, int64_t ldc,
               int out_mode, int64_t cutoff) {
  const int64_t m = A.rows, k = A.cols, n = B.cols;
  if (!splittable(m, k, n, cutoff)) {
    pl.leaves.push_back(make_desc(A, B, C, ldc, out_mode));
    return;
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
  for (int i = 0; i < 7; ++i) P[i] = alloc((size_t)(m0 * n0w));

  PreOp ps;
  ps.kind = 0;
  ps.in[0] = QView{A.p, A.ld, m0, k0w, ~0ull};
  ps.in[1] = QView{A.p + k0w, A.ld, m0, words(k1), tail_of(k1)};
  ps.in[2] = QView{A.p + m0 * A.ld, A.ld, m1, k0w, ~0ull};
  ps.in[3] = QView{A.p + m0 * A.ld + k0w, A.ld, m1, words(k1), tail_of(k1)};
  for (int i = 0; i < 4; ++i) ps.out[i] = S[i];
  ps.ldo = k0w; ps.R = m0; ps.Wd = k0w;
  pl.pre.push_back(ps);
  PreOp pt;
  pt.kind = 1;
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
  plan_node(pl, base, A_NW, B_NW, P[0], n0w, OUT_STORE, cutoff);   // P0 = A_NW B_NW
  plan_node(pl, base, A_NE, B_SW, P[1], n0w, OUT_STORE, cutoff);   // P1 = A_NE B_SW
  plan_node(pl, base, S3, B_SE, P[2], n0w, OUT_STORE, cutoff);     // P2 = S3 B_SE
  plan_node(pl, base, A_SE, T3, P[3], n0w, OUT_STORE, cutoff);     // P3 = A_SE T3
  plan_node(pl, base, S0, T0, P[4], n0w, OUT_STORE, cutoff);       // P4 = S0 T0
  plan_node(pl, base, S1, T1, P[5], n0w, OUT_STORE, cutoff);       // P5 = S1 T1
  plan_node(pl, base, S2, T2, P[6], n0w, OUT_STORE, cutoff);       // P6 = S2 T2

  PostOp po;
  for (int i = 0; i < 7; ++i) po.P[i] = P[i];
  po.ldp = n0w;
  po.c[0] = OView{C, ldc, m0, n0w, ~0ull};
  po.c[1] = OView{C + n0w, ldc, m0, words(n1), tail_of(n1)};
  po.c[2] = OView{C + m0 * ldc, ldc, m1, n0w, ~0ull};
  po.c[3] = OView{C + m0 * ldc + n0w, ldc, m1, words(n1), tail_of(n1)};
  po.mode = out_mode;
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

// Leaves of the product and the workspace they need: Strassen temporaries first, then
// the base kernel's scratch.  ``base`` == nullptr sizes only.
struct ProductPlan {
  StrassenPlan st;
  std::vector<MulDesc> leaves;   // when not recursing
  size_t scratch_words = 0;
  size_t total_words() const { return st.ws_words + scratch_words; }
};

void plan_product(ProductPlan& pp, uint64_t* base, uint64_t* C, int64_t ldc, const uint64_t* A, int64_t lda,
                  const uint64_t* B, int64_t ldb, int64_t m, int64_t k, int64_t n, bool accumulate,
                  const gf2_schedule& s) {
  const int out = accumulate ? OUT_XOR : OUT_STORE;
  const View Av{A, lda, m, k}, Bv{B, ldb, k, n};
  if (splittable(m, k, n, s.cutoff)) {
    plan_node(pp.st, base, Av, Bv, C, ldc, out, s.cutoff);
    pp.scratch_words = base_scratch_words(s, pp.st.leaves);
  } else {
    if (s.splitk > 1 && words(k) > 1) plan_splitk(pp.leaves, Av, Bv, C, ldc, s.splitk);
    else pp.leaves.push_back(make_desc(Av, Bv, C, ldc, out));
    pp.scratch_words = base_scratch_words(s, pp.leaves);
  }
}

size_t workspace_words(int64_t m, int64_t k, int64_t n, const gf2_schedule& s) {
  ProductPlan pp;
  plan_product(pp, nullptr, nullptr, words(n), nullptr, words(k), nullptr, words(n), m, k, n, false, s);
  return pp.total_words();
}

gf2_status execute(uint64_t* C, int64_t ldc, const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb,
                   int64_t m, int64_t k, int64_t n, bool accumulate, const gf2_schedule& s, hipStream_t st) {
  ProductPlan sizing;
  plan_product(sizing, nullptr, C, ldc, A, lda, B, ldb, m, k, n, accumulate, s);
  const size_t need = sizing.total_words() * 8;
  WorkspaceLease lease;
  gf2_status r = GF2_OK;
  if (need > 0 && (r = lease.acquire(need, st)) != GF2_OK) return r;
  uint64_t* ws = static_cast<uint64_t*>(lease.ptr());
  ProductPlan pp;
  plan_product(pp, ws, C, ldc, A, lda, B, ldb, m, k, n, accumulate, s);
  uint64_t* scratch = ws ? ws + pp.st.ws_words : nullptr;
  if (need > 0) lease.used();
  if (!pp.st.leaves.empty()) {
    for (const PreOp& p : pp.st.pre)
      if ((r = strassen_pre(p.kind, p.in, p.out, p.ldo, p.R, p.Wd, st)) != GF2_OK) return r;
    if ((r = run_base(s, pp.st.leaves, scratch, st)) != GF2_OK) return r;
    for (const PostOp& p : pp.st.post)   // children were pushed before their parent
      if ((r = strassen_post(p.P, p.ldp, p.c, p.mode, st)) != GF2_OK) return r;
    return GF2_OK;
  }
  if (s.splitk > 1 && words(k) > 1 && !accumulate)
    if ((r = fill_zero(OView{C, ldc, m, words(n), tail_of(n)}, st)) != GF2_OK) return r;
  return run_base(s, pp.leaves, scratch, st);
}

gf2_status mul_impl(uint64_t* C, int64_t ldc, const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb,
                    int64_t m, int64_t k, int64_t n, bool accumulate, const gf2_schedule* sched, void* stream) {
  g_err[0] = 0;
  gf2_status r = validate(C, ldc, A, lda, B, ldb, m, k, n);
  if (r != GF2_OK) return r;
  if ((r = validate_sched(sched)) != GF2_OK) return r;
  if (m == 0 || n == 0) return GF2_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (k == 0) return accumulate ? GF2_OK : fill_zero(OView{C, ldc, m, words(n), tail_of(n)}, st);
  const gf2_schedule s = resolve(sched, m, k, n);
  return execute(C, ldc, A, lda, B, ldb, m, k, n, accumulate, s, st);
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
  const gf2_schedule s = resolve(sched, m, k, n);
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
  for (auto& d : g_dev) {
    std::lock_guard<std::mutex> g(d.mu);
    if (d.base) (void)hipFree(d.base);
    if (d.last) (void)hipEventDestroy(d.last);
    d.base = nullptr;
    d.bytes = 0;
    d.last = nullptr;
    d.has_last = false;
  }
}

}  // extern "C"
