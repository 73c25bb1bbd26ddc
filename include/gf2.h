/*
 * gf2.h -- dense matrix multiplication over GF(2) on AMD MI355X (gfx950).
 *
 * The operation (Sections 1 and 2.3 of Albrecht, Bard and Hart, "Efficient
 * Multiplication of Dense Matrices over GF(2)"): for A (m x k) and B (k x n)
 * over the field with two elements, where addition is XOR and multiplication
 * is AND,
 *
 *     C[i][j] = XOR over t < k of (A[i][t] AND B[t][j]).
 *
 * It is computed by Strassen-Winograd recursion (Section 4, Algorithm 4) over a
 * Method of the Four Russians base case (Section 3, Algorithms 1-3), or over an
 * exact int8 matrix-core base case, or a popcount base case, chosen per call.
 * Every schedule gives the same bits: the result is unique and exact.
 *
 * LAYOUT (Section 2.1, "flat row-major"): a matrix with `rows` rows and `cols`
 * columns is `rows` rows of `ld` 64-bit words, ld >= ceil(cols/64).  Column j
 * of a row is bit (j & 63) of word (j >> 6) (least significant bit first).
 *   - Bits at columns >= cols in a row's last word are padding.  Inputs'
 *     padding is ignored.  gf2_mul writes C's padding as 0; gf2_addmul leaves
 *     it unchanged.
 *   - Words ceil(cols/64) .. ld-1 of a row (the stride gap) are never
 *     written and never affect the result.  Kernels may read the gap of an A
 *     or B row that has a later row (the bytes lie inside the matrix); they
 *     never read past the last row's last valid word.
 *   - Dimensions are in entries (bits); ld is in words.
 *
 * MEMORY AND OWNERSHIP.  A, B and C are device pointers (8-byte aligned) owned
 * by the caller, on the current HIP device.  C must not overlap A or B.  The
 * library owns a per-device workspace (Strassen temporaries, split-K partials,
 * descriptor staging), cached schedules and the schedule model; gf2_shutdown()
 * releases them.
 *
 * STREAMS.  `stream` is a hipStream_t (NULL = the null stream).  Calls enqueue
 * work and return without waiting, like BLAS; buffers must stay valid until the
 * stream reaches the work.  Workspace use is ordered across streams with events.
 *
 * ERRORS.  Arguments are validated before anything is enqueued; on error
 * nothing is enqueued and C is untouched.  A failed launch returns
 * GF2_ERR_DEVICE; gf2_last_error() gives the text (thread-local).  Faults in
 * kernels surface at the caller's next synchronisation.
 */
#ifndef GF2_H
#define GF2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gf2_status {
  GF2_OK = 0,
  GF2_ERR_INVALID_ARG = 1, /* negative size, short ld, null or misaligned pointer, bad schedule */
  GF2_ERR_ALIAS = 2,       /* C overlaps A or B (or two C's of a batch overlap) */
  GF2_ERR_ALLOC = 3,       /* device or host allocation failed */
  GF2_ERR_CAPTURE = 4,     /* would allocate while the stream is being captured */
  GF2_ERR_DEVICE = 5,      /* a HIP call or launch failed */
  GF2_ERR_UNSUPPORTED = 6  /* shape or option outside what the kernels handle */
} gf2_status;

/* Base-case kernels. */
enum {
  GF2_KERNEL_AUTO = 0,  /* library chooses */
  GF2_KERNEL_M4RM = 1,  /* Four Russians, Gray-code tables in LDS (Section 3) */
  GF2_KERNEL_MFMA = 2,  /* 0/1 int8 matrix-core product, low bit of the int32 sum */
  GF2_KERNEL_CUBIC = 3  /* AND + popcount parity against B transposed (Section 2.3) */
};

/* Odd sizes inside Strassen-Winograd (Section 4).  PAD: every split is at a word
 * border and the missing rows/columns of the smaller halves are treated as zero
 * (nothing is copied).  PEEL: each recursion node recurses on its largest part with
 * an even row count and k, n multiples of 128, and adds the peeled rows, columns and
 * inner slice with non-recursive base-case products. */
enum { GF2_ODD_PAD = 0, GF2_ODD_PEEL = 1 };

/* Workspace plan of Strassen-Winograd (Section 4).  FAST: every node's temporaries
 * (S0..S3, T0..T3, P0..P6) exist at once and all leaves of the product run in one launch.
 * LOW: at the top level, the memory-efficient schedule with two temporaries X (m/2 x
 * max(k, n)/2) and Y (k/2 x n/2): the seven products run one after another, written
 * straight into C's quadrants (each computed FAST below), with the additions between
 * them.  LOW applies to C := A*B with m even and n a multiple of 128; other calls run FAST. */
enum { GF2_MEM_FAST = 0, GF2_MEM_LOW = 1 };

/* A schedule: which base kernel, its tile variant, the Strassen-Winograd
 * crossover, the number of k slices, the odd-size rule, the M4RM table width
 * and the workspace plan.  Zero fields mean "default". */
typedef struct gf2_schedule {
  int32_t kernel;   /* GF2_KERNEL_* */
  int32_t variant;  /* kernel tile variant (see gf2_kernel_variants) */
  int32_t cutoff;   /* recurse while min(m, k, n) > cutoff; 0 = no recursion (Section 5, c_o) */
  int32_t splitk;   /* k split into this many slices XOR-combined into C; 0 or 1 = none */
  int32_t odd;      /* GF2_ODD_PAD or GF2_ODD_PEEL (only with cutoff > 0) */
  int32_t kappa;    /* M4RM table width k of Section 3.1 (index bits per Gray-code table):
                     * 0 = 8; 4..7 for the tiles of at most 1024 rows (variants 1-4, 12, 13,
                     * 18-20; others give GF2_ERR_UNSUPPORTED).  With kappa < 8 each base-case
                     * product first writes its A's kappa-bit fields out as bytes into the
                     * workspace; k must stay below kappa * 2^23. */
  int32_t memory;   /* GF2_MEM_FAST or GF2_MEM_LOW (only with cutoff > 0) */
} gf2_schedule;

/* C := A*B.  Section 1 / Section 2.3 definition above.  m, k, n >= 0.
 * k = 0 sets C's valid bits to 0; m = 0 or n = 0 does nothing. */
gf2_status gf2_mul(uint64_t* C, int64_t ldc, const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb,
                   int64_t m, int64_t k, int64_t n, void* stream);

/* C := C + A*B (XOR-accumulate).  Same arguments as gf2_mul; k = 0 does nothing. */
gf2_status gf2_addmul(uint64_t* C, int64_t ldc, const uint64_t* A, int64_t lda, const uint64_t* B,
                      int64_t ldb, int64_t m, int64_t k, int64_t n, void* stream);

/* gf2_mul / gf2_addmul (accumulate != 0) with an explicit schedule.  `sched`
 * may be NULL (library chooses).  Used by the autotuner and the tests. */
gf2_status gf2_mul_sched(uint64_t* C, int64_t ldc, const uint64_t* A, int64_t lda, const uint64_t* B,
                         int64_t ldb, int64_t m, int64_t k, int64_t n, int32_t accumulate,
                         const gf2_schedule* sched, void* stream);

/* gf2_mul_sched for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The
 * workspace (Strassen-Winograd temporaries, the base kernel's scratch) is a
 * static device array of GF2_NOALLOC_SCRATCH_BYTES that the library holds on
 * each GPU it runs on until the process ends; the call allocates no device
 * memory and does not synchronise.  Under GF2_POLICY_AUTOTUNE a shape missing
 * from the autotune cache takes the library's default schedule (nothing is
 * timed).  A schedule whose workspace (gf2_workspace_bytes) exceeds the array
 * gives GF2_ERR_UNSUPPORTED before anything is enqueued; pass a schedule with
 * fewer Strassen-Winograd levels (cutoff 0 needs none for the M4RM kernel).
 * Every call on one GPU uses that GPU's one array, so calls whose work overlaps
 * in time on one GPU (other streams, other threads) race and give wrong results:
 * order them, for instance on one stream. */
#define GF2_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
gf2_status gf2_mul_noalloc(uint64_t* C, int64_t ldc, const uint64_t* A, int64_t lda, const uint64_t* B,
                           int64_t ldb, int64_t m, int64_t k, int64_t n, int32_t accumulate,
                           const gf2_schedule* sched, void* stream);

/* The fixed list of candidate schedules that the autotuner and the schedule model
 * choose from (the batched executor's per-product choices).  gf2_candidate copies
 * entry `index` into *out. */
int32_t gf2_num_candidates(void);
gf2_status gf2_candidate(int32_t index, gf2_schedule* out);

/* ---- Batched products ----
 * Many independent products in one go: the base-case tiles of every product run in
 * one persistent kernel that pulls tiles (longest first) from an atomic queue;
 * Strassen-Winograd pre/post passes and split-K zero fills are separate kernels
 * around it, and products whose schedule is not a persistent-kernel variant run in
 * grouped launches beside it.  gf2_mul_batched captures this sequence in a HIP
 * graph on first sight of a batch (keyed by every pointer, shape and schedule) and
 * replays the graph afterwards. */
typedef struct gf2_problem {
  const uint64_t* A;
  const uint64_t* B;
  uint64_t* C;
  int64_t m, k, n;
  int64_t lda, ldb, ldc;
  int32_t accumulate; /* 0: C := A*B, 1: C := C + A*B */
  int32_t schedule;   /* index into the candidate list, or -1: library chooses */
} gf2_problem;

/* `probs` is a host array of `count` problems (copied).  Every problem is validated
 * as gf2_mul validates its arguments; in addition no C may overlap another product's
 * C, A or B (A and B may be shared).  On error nothing is enqueued. */
gf2_status gf2_mul_batched(const gf2_problem* probs, int64_t count, void* stream);

/* Explicit plans: create (validates, chooses schedules, allocates and uploads the
 * descriptors and workspace; synchronous), execute (enqueues launches only, no
 * allocation or host synchronisation, so it may be captured), destroy. */
typedef struct gf2_batch_plan_s* gf2_batch_plan;
gf2_status gf2_batch_plan_create(const gf2_problem* probs, int64_t count, gf2_batch_plan* out);
gf2_status gf2_batch_plan_execute(gf2_batch_plan plan, void* stream);
gf2_status gf2_batch_plan_destroy(gf2_batch_plan plan);
/* Schedule index chosen for problem i of the plan (-1 on bad arguments). */
int32_t gf2_batch_plan_schedule(gf2_batch_plan plan, int64_t i);

/* ---- Schedule policy, autotuner, schedule model ----
 * How the library chooses a schedule when the caller gives none:
 *   GF2_POLICY_FIXED    the built-in cost model: the M4RM tile, Strassen-Winograd cutoff and k
 *                       split of lowest predicted time (tile height against table-build
 *                       cost, Sections 3.2 and 5), or the streamed popcount for n <= 8;
 *                       batches use the tallest persistent-kernel tile by the same trade-off;
 *   GF2_POLICY_AUTOTUNE time every candidate once per shape bucket (powers of 2^(1/2)
 *                       of m, k, n), cache the fastest; falls back to FIXED under capture;
 *   GF2_POLICY_MODEL    the schedule model set by gf2_set_model: a single product takes the
 *                       argmin of its predicted log runtimes (latency head); a batch product
 *                       takes the batch head's argmin only where it is predicted at least 10%
 *                       faster than the FIXED candidate, else the FIXED candidate (the model's
 *                       outputs are natural-log milliseconds); falls back to FIXED when no model
 *                       is set.
 * Every schedule gives the same bits; the policy only changes the speed. */
enum { GF2_POLICY_FIXED = 0, GF2_POLICY_AUTOTUNE = 1, GF2_POLICY_MODEL = 2 };
gf2_status gf2_set_policy(int32_t policy);
int32_t gf2_get_policy(void);

/* Time every candidate schedule on an m x k by k x n product whose operands the
 * library fills with Bernoulli(density) bits on the device.  ms[i] (if not NULL,
 * gf2_num_candidates() entries) receives the median of `reps` timed runs after one
 * warm-up (a candidate that cannot run gets a negative value); *best the fastest
 * index.  Synchronises the device.  The result also enters the autotune cache. */
gf2_status gf2_autotune(int64_t m, int64_t k, int64_t n, double density, int32_t reps, float* ms, int32_t* best);
/* Throughput timing: the per-product time of each candidate when R copies of the product
 * (each with its own A, B and C, as in a real batch; R chosen so one batch holds enough work
 * to fill the GPU, with at most 512 MiB of operands, returned in *copies) run as one batch plan.  This is the cost that matters inside
 * gf2_mul_batched.  ms as in gf2_autotune; candidates are timed in batch form even when
 * they are not persistent-kernel schedules (they then run as grouped launches). */
gf2_status gf2_autotune_batch(int64_t m, int64_t k, int64_t n, double density, int32_t reps, float* ms,
                              int32_t* best, int32_t* copies);
/* Partial re-timing, for refreshing a timing set after a kernel change: as gf2_autotune
 * (batch == 0) or gf2_autotune_batch (batch != 0), but only the `count` candidates listed in
 * `candidates` (indices into the candidate list, in any order) are timed; ms[c] of every other
 * candidate is set to -1 (ms holds gf2_num_candidates() floats).  *copies (may be NULL)
 * receives the batch's copy count (1 for batch == 0).  The result does not enter the
 * autotune cache.  GF2_ERR_INVALID_ARG for an index outside [0, gf2_num_candidates()),
 * count < 0, candidates NULL with count > 0, or a density outside [0, 1], checked before
 * any device work. */
gf2_status gf2_autotune_candidates(int64_t m, int64_t k, int64_t n, double density, int32_t reps, int32_t batch,
                                   const int32_t* candidates, int32_t count, float* ms, int32_t* copies);
/* Autotune cache persistence (text file: one "m_bucket k_bucket n_bucket index" line per entry). */
gf2_status gf2_autotune_save(const char* path);
gf2_status gf2_autotune_load(const char* path);
void gf2_autotune_clear(void);

/* ---- Schedule model kernels ----
 * A float32 MLP: 4 inputs (log2 m, log2 k, log2 n, density, each standardised) ->
 * three hidden layers of 64 with ReLU -> 2 * gf2_num_candidates() outputs: the predicted
 * (standardised) log runtimes of the candidate schedules for a product on its own
 * (outputs 0 .. S-1, used by gf2_mul) and per product inside a batch (outputs S .. 2S-1,
 * used by batch plans; see gf2_autotune_batch).  Parameters are one flat
 * float array, layer by layer, W (fan_in x fan_out, row-major) then b.  All pointers
 * below are device pointers; X is batch x 4, Y and T and M are batch x outputs.
 * acts: 3 * batch * 64 floats (pre-activations, written by forward, read by
 * backward); scratch: gf2_mlp_scratch_floats(batch) floats.  The loss is the mean
 * over observed entries (M = 1) of (Y - T)^2; grads receives its gradient.  Adam
 * follows Kingma and Ba with bias correction; `step` counts from 1.  Reductions run
 * in a fixed order, so results are reproducible. */
int64_t gf2_mlp_param_count(void);
int64_t gf2_mlp_scratch_floats(int64_t batch);
gf2_status gf2_mlp_forward(const float* params, const float* X, int64_t batch, float* Y, float* acts, void* stream);
gf2_status gf2_mlp_backward(const float* params, const float* X, int64_t batch, const float* acts, const float* Y,
                            const float* T, const float* M, float* grads, float* scratch, float* loss, void* stream);
gf2_status gf2_mlp_adam(float* params, const float* grads, float* m, float* v, int64_t count, int32_t step, float lr,
                        float beta1, float beta2, float eps, void* stream);
/* out[b] = argmin over allowed outputs of Y[b] (allowed: device mask of the 2S outputs, or NULL for all). */
gf2_status gf2_mlp_argmin(const float* Y, int64_t batch, const uint8_t* allowed, int32_t* out, void* stream);
/* Install the schedule model used by GF2_POLICY_MODEL: host arrays, copied.  norm holds
 * the mean[4] then std[4] of the raw features (log2 m, log2 k, log2 n, density).
 * count must equal gf2_mlp_param_count().  NULL params removes the model. */
gf2_status gf2_set_model(const float* params, int64_t count, const float* norm);
/* Candidate the current policy picks for a product of this shape (batch != 0: only
 * schedules the persistent kernel can run). */
int32_t gf2_choose_schedule(int64_t m, int64_t k, int64_t n, int32_t batch);
/* The schedule gf2_mul_sched(..., req, ...) runs for a product of this shape under the
 * current policy; req NULL is the library's own choice (under GF2_POLICY_FIXED the M4RM
 * tile height, Strassen-Winograd cutoff and k split of lowest predicted time, Section 5).
 * Under GF2_POLICY_AUTOTUNE this may time the candidates first.  *out is written on
 * GF2_OK; negative dimensions, a NULL out or an invalid req give GF2_ERR_INVALID_ARG. */
gf2_status gf2_resolve_schedule(int64_t m, int64_t k, int64_t n, const gf2_schedule* req, gf2_schedule* out);

/* Number of tile variants of a base kernel (0 for an unknown kernel). */
int32_t gf2_kernel_variants(int32_t kernel);

/* Device workspace, in bytes, that C := A*B of this shape under `sched` uses
 * (Strassen temporaries, narrow-table index bytes, base-kernel scratch; 0 when
 * none).  C := C + A*B always plans GF2_MEM_FAST: size it with memory = FAST. */
size_t gf2_workspace_bytes(int64_t m, int64_t k, int64_t n, const gf2_schedule* sched);

/* Grow the current device's workspace to at least `bytes` now (synchronising
 * the device), so that later calls -- for instance under stream capture --
 * need no allocation.  A call made under stream capture records the
 * workspace's address into the graph; from then on the library never frees
 * that buffer before gf2_shutdown(): a later, larger eager call allocates a
 * new buffer and keeps the captured one, so the graph stays valid to replay
 * (while no other call on the device uses the workspace at the same time).
 * Replaying such a graph after gf2_shutdown() is invalid. */
gf2_status gf2_reserve_workspace(size_t bytes);

/* ---- Launch tracing (for measurement; off by default) ----
 * While enabled, the library brackets every kernel launch with a pair of HIP
 * events on the launch's stream and records the kernel kind and its
 * algorithmic work.  gf2_trace_read synchronises those events.  Not for use
 * under stream capture. */
enum {
  GF2_TRACE_M4RM = 1,   /* work = 64-bit table-row additions m*ceil(k/8)*ceil(n/64) */
  GF2_TRACE_MFMA = 2,   /* work = multiply-accumulates m*k*n */
  GF2_TRACE_CUBIC = 3,  /* work = 64-bit AND+popcount steps m*n*ceil(k/64) */
  GF2_TRACE_PRE = 4,    /* work = bytes moved by the Strassen pre-additions */
  GF2_TRACE_POST = 5,   /* work = bytes moved by the Strassen post-additions */
  GF2_TRACE_FILL = 6,   /* work = bytes written */
  GF2_TRACE_BATCH = 7   /* work = 64-bit table-row additions of a batched launch */
};
typedef struct gf2_trace_record {
  int32_t kind;    /* GF2_TRACE_* */
  int32_t items;   /* products (or passes) in the launch */
  double work;     /* algorithmic work of the launch, unit per kind */
  double ms;       /* launch duration from its event pair */
} gf2_trace_record;
gf2_status gf2_trace_enable(int32_t on);
/* Copies up to `max` records (oldest first) into `out` and sets *count to the number
 * copied; synchronises the recorded events.  Records stay until gf2_trace_clear. */
gf2_status gf2_trace_read(gf2_trace_record* out, int64_t max, int64_t* count);
void gf2_trace_clear(void);

/* ---- LDS bandwidth probe (measurement only) ----
 * The ceiling against which the M4RM kernels' table traffic is reported: their lookups
 * (Section 3, AddRowFromTable) read LDS and their table builds (MakeTable) write it.
 * Launches `blocks` workgroups of 1024 threads on `stream`; each issues iters x 64
 * conflict-free LDS accesses per thread in the four-table tile's pattern: mode 0 reads
 * 16 B per lane (ds_read_b128), mode 1 writes 4 B per lane (ds_write_b32, whole 256 B
 * table entries as the Gray-code build writes them).  `out` is a device buffer of
 * blocks x 1024 words (caller-owned) that receives a reduction of what was read, so no
 * access can be elided.  *bytes (if not NULL) receives the LDS bytes the launch moves.
 * Time the launch with events on `stream`.  Bad arguments give GF2_ERR_INVALID_ARG. */
gf2_status gf2_lds_probe(int32_t mode, int32_t blocks, int32_t iters, uint64_t* out, double* bytes, void* stream);

const char* gf2_status_string(gf2_status s);
/* Text of the last error raised on the calling thread ("" if none). */
const char* gf2_last_error(void);

/* Release every device and host resource the library holds, on all devices. */
void gf2_shutdown(void);

#ifdef __cplusplus
}
#endif

#endif /* GF2_H */
