// Internal declarations shared by the library's translation units.
// Not part of the public ABI (that is include/gf2.h).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>
#include <vector>
#include "gf2.h"

namespace gf2 {

// How a kernel writes its result tile into C.
enum OutMode : int32_t {
  OUT_STORE = 0,    // C := P            (padding bits written 0)
  OUT_XOR = 1,      // C := C ^ P        (non-atomic read-modify-write; padding unchanged)
  OUT_ATOMIC = 2,   // C ^= P atomically (several producers of the same C words)
};

// One product C (m x n) <- A (m x k) * B (k x n), each a window of a row-major packed
// matrix: ``ld`` words per row, column j of a row at bit j&63 of word j>>6.
struct MulDesc {
  const uint64_t* A;
  const uint64_t* B;
  uint64_t* C;
  int64_t lda, ldb, ldc;
  int32_t m, k, n;
  int32_t out;        // OutMode
};

__host__ __device__ inline int64_t words(int64_t bits) { return (bits + 63) >> 6; }

// Error reporting (thread-local text, read back through gf2_last_error()).
gf2_status set_error(gf2_status s, const char* fmt, ...);
gf2_status hip_check(hipError_t e, const char* what);

// Launch tracing: bracket a launch with events when tracing is on.
class TraceScope {
 public:
  TraceScope(int kind, int items, double work, hipStream_t s);
  ~TraceScope();
 private:
  int kind_, items_;
  double work_;
  hipStream_t s_;
  hipEvent_t e0_ = nullptr;
};
bool trace_on();
void trace_suspend(bool on);   // no event records while a graph is being captured

// Candidate schedules (sched.cpp).
int num_candidates();
const gf2_schedule& candidate(int i);
// Candidate index for a product when the caller leaves the choice to the library,
// under the current policy (fixed heuristic, autotune cache, or schedule model).
// ``batch`` restricts the choice to schedules the persistent kernel can run.
// ``may_time`` false: no autotune timing (a shape missing from the cache falls back).
int choose_candidate(int64_t m, int64_t k, int64_t n, bool batch, hipStream_t s, bool may_time = true);
int fixed_candidate(int64_t m, int64_t k, int64_t n);
// Schedule model inference on the host copy of the weights: predicted log runtimes.
bool model_predict(int64_t m, int64_t k, int64_t n, double density, float* out);
bool model_available();
// Batch schedules under the model policy: the model's candidate replaces the fixed rule's
// only where it is predicted at least this fraction faster (smaller predicted gains are within
// the model's error, and end to end they cost more than they save).
constexpr double kModelBatchMargin = 0.10;
int model_or_fixed(int pick, float y_pick, int fixed, float y_fixed);
gf2_status model_choose_batch(const std::vector<float>& feats_raw, const uint8_t* allowed_host,
                              const std::vector<int>& fixed, std::vector<int>& out);
bool batch_allowed(int candidate);
void bump_policy_epoch();   // invalidates cached batch plans after a policy or model change

// A product computed in a workspace the caller provides instead of the library's arena:
// validates, resolves the schedule without autotune timing, and rejects a schedule whose
// workspace exceeds ``max_bytes`` with GF2_ERR_UNSUPPORTED before anything is enqueued.
// ``scratch`` returns the workspace's device address for the current device.  Allocates no
// device memory.
using ScratchFn = gf2_status (*)(uint64_t** out);
gf2_status mul_in_static(uint64_t* C, int64_t ldc, const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb,
                         int64_t m, int64_t k, int64_t n, bool accumulate, const gf2_schedule* sched, void* stream,
                         size_t max_bytes, ScratchFn scratch);

// ---- kernels (each .hip file owns its launches) ----
// Products launched together with descriptors passed by value in the kernel arguments.
constexpr int kMaxGroup = 56;   // 7^2 Strassen leaves plus a k-split tail (fits 4 KiB of kernel arguments)
struct GroupArgs {
  MulDesc d[kMaxGroup];
  int tile_start[kMaxGroup + 1];
  int count;
  int remap_n;   // workgroups [0, remap_n) use the XCD remap; later ones (a short tail) map 1:1
};

// M4RM base case (m4rm.hip).  Table width ``kappa`` (index bits per table) is 8 for every
// tile and 4..7 for the tiles m4rm_has_kappa names; a descriptor launched with kappa < 8 has
// its A replaced by A's index expansion (m4rm_expand).
int m4rm_num_variants();
int m4rm_tile_rows(int variant);
int m4rm_phase_rows(int variant, int kappa = 8);   // rows of B consumed per table-build phase
int m4rm_tile_words(int variant);
bool m4rm_has_kappa(int variant, int kappa);
int64_t m4rm_tiles(const MulDesc& d, int variant);
// The last ``tail`` descriptors (short k slices) are dispatched after all others, outside
// the XCD remap, so they fill the last round of tiles.
gf2_status m4rm_launch_group(const MulDesc* descs, int count, int variant, hipStream_t s, int tail = 0,
                             int kappa = 8);
// Index expansion for tables of kappa < 8 bits: byte j of row r of X = bits kappa*j ..
// kappa*j + kappa - 1 of row r of A (bits at or past k as zero); X has ldx words per row,
// ldx = m4rm_expanded_ld(k, kappa), and bytes past ceil(k/kappa) are zero.
struct ExpandOp {
  const uint64_t* A;
  uint64_t* X;
  int64_t lda, ldx;
  int32_t m, k, kappa, pad;
};
int64_t m4rm_expanded_ld(int64_t k, int kappa);
gf2_status m4rm_expand(const ExpandOp* ops, int n, hipStream_t s);                          // host array
gf2_status m4rm_expand_list(const ExpandOp* dev_ops, int n, int64_t max_dwords, hipStream_t s);  // device array
// One queue item of the persistent batch kernel: a C tile of descriptor ``desc``; ``variant``
// holds the tile variant in bits 0-7 and the table width above.
struct BatchItem {
  int32_t desc, tm, tn, variant;
};
bool m4rm_batchable(int variant);   // can run inside the persistent kernel
gf2_status m4rm_launch_persistent(const MulDesc* dev_descs, const BatchItem* dev_items, int nitems, int* dev_counter,
                                  int grid, hipStream_t s);

// Exact int8 matrix-core base case (mfma.hip).  Each product's B is first transposed into
// scratch (transpose_words each, one after another).
int64_t mfma_tiles(const MulDesc& d);
gf2_status mfma_launch_group(const MulDesc* descs, int count, uint64_t* scratch, hipStream_t s);

// Popcount base case with B transposed into scratch (cubic.hip).
size_t cubic_scratch_words(const MulDesc& d);
// Words of B transposed into 64 x 64 bit blocks (transpose_launch), as the int8 matrix-core
// base reads it: every product of a grouped launch keeps a slice of this size.
size_t transpose_words(const MulDesc& d);
gf2_status cubic_launch(const MulDesc& d, uint64_t* scratch, hipStream_t s);
// True when the popcount base case streams A against n <= 8 columns of B held in LDS.
bool cubic_narrow(const MulDesc& d);
bool cubic_narrow_shape(int64_t k, int64_t n);
// B (k x n) into bt in k-word-major order: bt[w * 64*words(n) + j] = bits 64w..64w+63 of
// column j; rows >= k read as zero.
gf2_status transpose_launch(const MulDesc& d, uint64_t* bt, hipStream_t s);

// Schedule model kernels (mlp.hip).
int64_t mlp_param_count(int nout);
int64_t mlp_scratch_floats(int64_t batch, int nout);
gf2_status mlp_forward(const float* params, const float* X, int64_t batch, int nout, float* Y, float* acts,
                       hipStream_t s);
gf2_status mlp_backward(const float* params, const float* X, int64_t batch, int nout, const float* acts,
                        const float* Y, const float* T, const float* M, float* grads, float* scratch, float* loss,
                        hipStream_t s);
gf2_status mlp_adam(float* p, const float* g, float* m, float* v, int64_t n, int32_t step, float lr, float b1,
                    float b2, float eps, hipStream_t s);
gf2_status mlp_argmin(const float* Y, int64_t batch, int nout, const uint8_t* allowed, int32_t* out, hipStream_t s);
void mlp_forward_host(const float* params, const float* x, int nout, float* y);

// Element-wise XOR passes (xorops.hip).
// A window of a packed matrix with virtual zero padding: rows >= rows and words >= wds
// read as zero; the word wds-1 is ANDed with ``tail``.
struct QView {
  const uint64_t* p;
  int64_t ld;
  int64_t rows, wds;
  uint64_t tail;
};
struct OView {
  uint64_t* p;
  int64_t ld;
  int64_t rows, wds;   // region actually written
  uint64_t tail;       // mask for word wds-1 (padding bits written 0 or left unchanged)
};
gf2_status fill_zero(const OView& o, hipStream_t s);
// o := a XOR b over o's region (o may be a or b); traced as ``trace_kind``.
gf2_status xor2(const OView& o, const QView& a, const QView& b, int trace_kind, hipStream_t s);
// Strassen-Winograd passes of one recursion node (``depth`` 0 = the root), Algorithm 4.
// Pre-additions: from the quadrants NW, NE, SW, SE of A (kind 0) produce S0..S3, of B
// (kind 1) T0..T3, over R x Wd words.  Post-additions: from P0..P6 (ld ldp) write the
// four quadrants of C.
struct PreOp {
  int32_t kind;        // 0: S0..S3 from A's quadrants; 1: T0..T3 from B's
  int32_t depth;
  QView in[4];         // NW, NE, SW, SE
  uint64_t* out[4];
  int64_t ldo, R, Wd;
};
struct PostOp {
  int32_t mode;        // OutMode for C
  int32_t depth;
  const uint64_t* P[7];
  int64_t ldp;
  OView c[4];          // C_NW, C_NE, C_SW, C_SE
};
// Two recursion levels in one pass (a node and its seven children, every split exact: all
// operands are 4 x 4 blocks of R4 x W4-word sub-quadrants).  Pre: from ``in`` (A for kind 0,
// B for kind 1) the node's four S (T) into ``node`` and child c's four S' (T') into child[c].
struct Pre2Op {
  int32_t kind;
  const uint64_t* in;
  int64_t ldi, R4, W4;
  uint64_t* node[4];
  int64_t ldn;
  uint64_t* child[7][4];
  int64_t ldc;
};
struct Pre2Args {
  Pre2Op op[2];
};
// Post: from child c's leaf products P[c][0..6] (ld ldp) the node's C (mode OUT_STORE or OUT_XOR).
struct Post2Op {
  int32_t mode;
  const uint64_t* P[7][7];
  int64_t ldp;
  uint64_t* C;
  int64_t ldc, R4, W4;
};
gf2_status strassen_pre2(const Pre2Op& a_side, const Pre2Op& b_side, hipStream_t s);
gf2_status strassen_post2(const Post2Op& a, hipStream_t s);
// Many independent ops in one launch (device arrays); max_elems = largest op's word count.
gf2_status fill_zero_multi(const OView* dev_ops, int n, int64_t max_elems, hipStream_t s);
gf2_status strassen_pre_multi(const PreOp* dev_ops, int n, int64_t max_elems, hipStream_t s);
gf2_status strassen_post_multi(const PostOp* dev_ops, int n, int64_t max_elems, hipStream_t s);
// Host arrays of ops that may run concurrently (one recursion depth), launched kArgOps at
// a time with the ops as kernel arguments.
constexpr int kArgOps = 16;
gf2_status strassen_pre_ops(const PreOp* ops, int n, hipStream_t s);
gf2_status strassen_post_ops(const PostOp* ops, int n, hipStream_t s);
gf2_status fill_random(uint64_t* p, int64_t nwords, uint64_t seed, double density, hipStream_t s);

}  // namespace gf2
