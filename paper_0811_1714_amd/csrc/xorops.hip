// Element-wise passes over packed GF(2) matrices: bulk zeroing and the fused
// pre- and post-additions of Strassen-Winograd (Section 4, Algorithm 4).
// Over GF(2) addition and subtraction are both XOR (Section 2.2: a row addition
// is a word-wise XOR).  These passes are bound by HBM bandwidth: each thread
// handles one 64-bit word position, consecutive threads consecutive words.
#include "gf2_internal.h"

namespace gf2 {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ uint64_t qload(const QView& v, int64_t r, int64_t w) {
  if (r >= v.rows || w >= v.wds) return 0;
  uint64_t x = v.p[r * v.ld + w];
  return w == v.wds - 1 ? (x & v.tail) : x;
}

__device__ __forceinline__ void owrite(const OView& o, int64_t r, int64_t w, uint64_t x, int mode) {
  if (r >= o.rows || w >= o.wds) return;
  if (w == o.wds - 1) x &= o.tail;
  uint64_t* p = o.p + r * o.ld + w;
  *p = mode == OUT_STORE ? x : (*p ^ x);
}

__global__ void fill_zero_kernel(OView o) {
  const int64_t total = o.rows * o.wds;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / o.wds, w = i - r * o.wds;
    o.p[r * o.ld + w] = 0;
  }
}

// kind 0 (A):  S0 = SW+SE, S1 = S0+NW, S2 = NW+SW, S3 = NE+S1
// kind 1 (B):  T0 = NE+NW, T1 = SE+T0, T2 = SE+NE, T3 = T1+SW
__device__ __forceinline__ void pre_element(const PreOp& a, int64_t i) {
  const int64_t r = i / a.Wd, w = i - r * a.Wd;
  const uint64_t nw = qload(a.in[0], r, w), ne = qload(a.in[1], r, w);
  const uint64_t sw = qload(a.in[2], r, w), se = qload(a.in[3], r, w);
  uint64_t o0, o1, o2, o3;
  if (a.kind == 0) {
    o0 = sw ^ se;
    o1 = o0 ^ nw;
    o2 = nw ^ sw;
    o3 = ne ^ o1;
  } else {
    o0 = ne ^ nw;
    o1 = se ^ o0;
    o2 = se ^ ne;
    o3 = o1 ^ sw;
  }
  const int64_t off = r * a.ldo + w;
  a.out[0][off] = o0;
  a.out[1][off] = o1;
  a.out[2][off] = o2;
  a.out[3][off] = o3;
}

__global__ void strassen_pre_multi_kernel(const PreOp* __restrict__ ops) {
  const PreOp a = ops[blockIdx.y];
  const int64_t total = a.R * a.Wd;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
    pre_element(a, i);
}

// U0 = P0+P1, U1 = P0+P5, U2 = U1+P6, U3 = U1+P4, U4 = U3+P2, U5 = U2+P3, U6 = U2+P4;
// C_NW = U0, C_NE = U4, C_SW = U5, C_SE = U6.  The grid covers C_NW's region, which
// contains the other three (top/left halves are the larger ones).
__device__ __forceinline__ void post_element(const PostOp& a, int64_t i) {
  const int64_t Wd = a.c[0].wds;
  const int64_t r = i / Wd, w = i - r * Wd;
  const int64_t off = r * a.ldp + w;
  const bool ne = r < a.c[1].rows && w < a.c[1].wds;
  const bool sw = r < a.c[2].rows && w < a.c[2].wds;
  const bool se = r < a.c[3].rows && w < a.c[3].wds;
  const uint64_t p0 = a.P[0][off];
  owrite(a.c[0], r, w, p0 ^ a.P[1][off], a.mode);
  if (ne || sw || se) {
    const uint64_t u1 = p0 ^ a.P[5][off];
    const uint64_t p4 = (ne || se) ? a.P[4][off] : 0;
    if (ne) owrite(a.c[1], r, w, u1 ^ p4 ^ a.P[2][off], a.mode);
    if (sw || se) {
      const uint64_t u2 = u1 ^ a.P[6][off];
      if (sw) owrite(a.c[2], r, w, u2 ^ a.P[3][off], a.mode);
      if (se) owrite(a.c[3], r, w, u2 ^ p4, a.mode);
    }
  }
}

__global__ void strassen_post_multi_kernel(const PostOp* __restrict__ ops) {
  const PostOp a = ops[blockIdx.y];
  const int64_t total = a.c[0].rows * a.c[0].wds;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
    post_element(a, i);
}

// Up to kArgOps ops of one recursion depth passed by value (no device staging, so a
// single product's passes need no host-to-device copy); blockIdx.y selects the op.
template <class Op>
struct OpBatch {
  int32_t count;
  Op op[kArgOps];
};

__global__ void strassen_pre_args_kernel(OpBatch<PreOp> b) {
  const PreOp& a = b.op[blockIdx.y];
  const int64_t total = a.R * a.Wd;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
    pre_element(a, i);
}

__global__ void strassen_post_args_kernel(OpBatch<PostOp> b) {
  const PostOp& a = b.op[blockIdx.y];
  const int64_t total = a.c[0].rows * a.c[0].wds;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
    post_element(a, i);
}

__global__ void fill_zero_multi_kernel(const OView* __restrict__ ops) {
  const OView o = ops[blockIdx.y];
  const int64_t total = o.rows * o.wds;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / o.wds, w = i - r * o.wds;
    o.p[r * o.ld + w] = 0;
  }
}

// out := a XOR b over out's region; a and b read as zero past their rows and words (the
// additions of Section 4's two-temporary schedule).  out may be a or b itself: each word is
// read before it is written, by the same thread.
__global__ void xor2_kernel(OView o, QView a, QView b) {
  const int64_t total = o.rows * o.wds;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / o.wds, w = i - r * o.wds;
    owrite(o, r, w, qload(a, r, w) ^ qload(b, r, w), OUT_STORE);
  }
}

// Two recursion levels of Algorithm 4 in one pass each, for a node whose quadrants and whose
// children's quadrants all split exactly (m a multiple of 4, k and n of 256): every operand is
// then a block of 4 x 4 equal sub-quadrants, X[i][j] = rows i*R4.., words j*W4...
//   pre:  from A's (B's) sixteen sub-quadrants, the node's S0..S3 (T0..T3) and every child's
//         S'0..S'3 (T'0..T'3), the child operands being {A_NW, A_NE, S3, A_SE, S0, S1, S2}
//         (B: {B_NW, B_SW, B_SE, T3, T0, T1, T2}) as in the products P0..P6;
//   post: from the 49 leaf products, each child's U0, U4, U5, U6 (its output's quadrants, i.e.
//         the node's P_c by sub-quadrant) and from those the node's C quadrants.
// A pass reads each input word once, so the node's own P0..P6 never go through memory.
__device__ __forceinline__ void s_of(int kind, const uint64_t (&q)[4], uint64_t (&o)[4]) {
  // q = NW, NE, SW, SE of one operand at one position; o = S0..S3 (kind 0) or T0..T3 (kind 1).
  if (kind == 0) {
    o[0] = q[2] ^ q[3];
    o[1] = o[0] ^ q[0];
    o[2] = q[0] ^ q[2];
    o[3] = q[1] ^ o[1];
  } else {
    o[0] = q[1] ^ q[0];
    o[1] = q[3] ^ o[0];
    o[2] = q[3] ^ q[1];
    o[3] = o[1] ^ q[2];
  }
}

// KIND (0: the A side, 1: the B side) is a template argument so that the child operands'
// sources below are compile-time indices: with a run-time kind the private arrays they index
// would live in scratch memory.
template <int KIND>
__device__ __forceinline__ void strassen_pre2_side(const Pre2Op& a) {
  const int64_t total = a.R4 * a.W4;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / a.W4, w = i - r * a.W4;
    uint64_t x[4][4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int bj = 0; bj < 4; ++bj) x[bi][bj] = a.in[(bi * a.R4 + r) * a.ldi + bj * a.W4 + w];
    // The node's quadrants by sub-position qi, qj, then its S (T), written by sub-position.
    uint64_t nodeq[4][4], st[4][4];   // [sub-position][NW, NE, SW, SE] and [sub-position][S0..S3]
#pragma unroll
    for (int qi = 0; qi < 2; ++qi)
#pragma unroll
      for (int qj = 0; qj < 2; ++qj) {
        const int sp = 2 * qi + qj;
        nodeq[sp][0] = x[qi][qj];
        nodeq[sp][1] = x[qi][2 + qj];
        nodeq[sp][2] = x[2 + qi][qj];
        nodeq[sp][3] = x[2 + qi][2 + qj];
        s_of(KIND, nodeq[sp], st[sp]);
#pragma unroll
        for (int t = 0; t < 4; ++t) a.node[t][(qi * a.R4 + r) * a.ldn + qj * a.W4 + w] = st[sp][t];
      }
    // Child operand c by sub-position: a node quadrant (index) or one of its S (T) (4 + index).
    constexpr int A_OPS[7] = {0, 1, 4 + 3, 3, 4 + 0, 4 + 1, 4 + 2};
    constexpr int B_OPS[7] = {0, 2, 3, 4 + 3, 4 + 0, 4 + 1, 4 + 2};
#pragma unroll
    for (int c = 0; c < 7; ++c) {
      const int src = KIND == 0 ? A_OPS[c] : B_OPS[c];
      uint64_t q[4], o[4];
#pragma unroll
      for (int sp = 0; sp < 4; ++sp) q[sp] = src < 4 ? nodeq[sp][src] : st[sp][src - 4];
      s_of(KIND, q, o);
#pragma unroll
      for (int t = 0; t < 4; ++t) a.child[c][t][r * a.ldc + w] = o[t];
    }
  }
}

__global__ void strassen_pre2_kernel(Pre2Args args) {
  const Pre2Op& a = args.op[blockIdx.y];
  if (a.kind == 0)
    strassen_pre2_side<0>(a);
  else
    strassen_pre2_side<1>(a);
}

__global__ void strassen_post2_kernel(Post2Op a) {
  const int64_t total = a.R4 * a.W4;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / a.W4, w = i - r * a.W4;
    const int64_t off = r * a.ldp + w;
    uint64_t v[7][4];   // child c's output by sub-position: U0 (NW), U4 (NE), U5 (SW), U6 (SE)
#pragma unroll
    for (int c = 0; c < 7; ++c) {
      uint64_t p[7];
#pragma unroll
      for (int j = 0; j < 7; ++j) p[j] = a.P[c][j][off];
      const uint64_t u1 = p[0] ^ p[5], u2 = u1 ^ p[6];
      v[c][0] = p[0] ^ p[1];
      v[c][1] = u1 ^ p[4] ^ p[2];
      v[c][2] = u2 ^ p[3];
      v[c][3] = u2 ^ p[4];
    }
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) {
      const int qi = sp >> 1, qj = sp & 1;
      const uint64_t u1 = v[0][sp] ^ v[5][sp], u2 = u1 ^ v[6][sp];
      const uint64_t out[4] = {v[0][sp] ^ v[1][sp], u1 ^ v[4][sp] ^ v[2][sp], u2 ^ v[3][sp], u2 ^ v[4][sp]};
#pragma unroll
      for (int Q = 0; Q < 4; ++Q) {
        const int Qi = Q >> 1, Qj = Q & 1;
        uint64_t* cp = a.C + ((2 * Qi + qi) * a.R4 + r) * a.ldc + (2 * Qj + qj) * a.W4 + w;
        *cp = a.mode == OUT_STORE ? out[Q] : (*cp ^ out[Q]);
      }
    }
  }
}

unsigned grid_for(int64_t total) {
  int64_t b = (total + kThreads - 1) / kThreads;
  const int64_t cap = 256 * 16;
  return (unsigned)(b < 1 ? 1 : (b > cap ? cap : b));
}

}  // namespace

gf2_status fill_zero(const OView& o, hipStream_t s) {
  if (o.rows <= 0 || o.wds <= 0) return GF2_OK;
  TraceScope trace(GF2_TRACE_FILL, 1, 8.0 * o.rows * o.wds, s);
  hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(o.rows * o.wds)), dim3(kThreads), 0, s, o);
  return hip_check(hipGetLastError(), "fill_zero launch");
}

gf2_status xor2(const OView& o, const QView& a, const QView& b, int trace_kind, hipStream_t s) {
  if (o.rows <= 0 || o.wds <= 0) return GF2_OK;
  TraceScope trace(trace_kind, 1, 24.0 * o.rows * o.wds, s);
  hipLaunchKernelGGL(xor2_kernel, dim3(grid_for(o.rows * o.wds)), dim3(kThreads), 0, s, o, a, b);
  return hip_check(hipGetLastError(), "xor2 launch");
}

gf2_status strassen_pre2(const Pre2Op& a_side, const Pre2Op& b_side, hipStream_t s) {
  Pre2Args args;
  args.op[0] = a_side;
  args.op[1] = b_side;
  const int64_t mx = std::max(a_side.R4 * a_side.W4, b_side.R4 * b_side.W4);
  if (mx <= 0) return GF2_OK;
  const double bytes = 8.0 * (a_side.R4 * a_side.W4 + b_side.R4 * b_side.W4) * (16 + 16 + 28);
  TraceScope trace(GF2_TRACE_PRE, 2, bytes, s);
  hipLaunchKernelGGL(strassen_pre2_kernel, dim3(grid_for(mx), 2), dim3(kThreads), 0, s, args);
  return hip_check(hipGetLastError(), "strassen_pre2 launch");
}

gf2_status strassen_post2(const Post2Op& a, hipStream_t s) {
  const int64_t total = a.R4 * a.W4;
  if (total <= 0) return GF2_OK;
  TraceScope trace(GF2_TRACE_POST, 1, 8.0 * total * (49 + 16 * (a.mode == OUT_STORE ? 1 : 2)), s);
  hipLaunchKernelGGL(strassen_post2_kernel, dim3(grid_for(total)), dim3(kThreads), 0, s, a);
  return hip_check(hipGetLastError(), "strassen_post2 launch");
}

// Multi-op launches: blockIdx.y selects the op; x blocks stride over its words.
unsigned multi_x(int64_t max_elems, int n) {
  int64_t b = (max_elems + kThreads - 1) / kThreads;
  const int64_t cap = n >= 64 ? 16 : 256 * 8 / (n > 0 ? n : 1);
  return (unsigned)(b < 1 ? 1 : (b > cap ? cap : b));
}

gf2_status strassen_pre_ops(const PreOp* ops, int n, hipStream_t s) {
  for (int base = 0; base < n; base += kArgOps) {
    OpBatch<PreOp> b;
    b.count = std::min(kArgOps, n - base);
    int64_t mx = 0;
    double bytes = 0;
    for (int i = 0; i < b.count; ++i) {
      b.op[i] = ops[base + i];
      mx = std::max(mx, b.op[i].R * b.op[i].Wd);
      bytes += 64.0 * b.op[i].R * b.op[i].Wd;
    }
    if (mx <= 0) continue;
    TraceScope trace(GF2_TRACE_PRE, b.count, bytes, s);
    hipLaunchKernelGGL(strassen_pre_args_kernel, dim3(multi_x(mx, b.count), b.count), dim3(kThreads), 0, s, b);
    gf2_status r = hip_check(hipGetLastError(), "strassen_pre_ops launch");
    if (r != GF2_OK) return r;
  }
  return GF2_OK;
}

gf2_status strassen_post_ops(const PostOp* ops, int n, hipStream_t s) {
  for (int base = 0; base < n; base += kArgOps) {
    OpBatch<PostOp> b;
    b.count = std::min(kArgOps, n - base);
    int64_t mx = 0;
    double bytes = 0;
    for (int i = 0; i < b.count; ++i) {
      b.op[i] = ops[base + i];
      const int64_t t = b.op[i].c[0].rows * b.op[i].c[0].wds;
      mx = std::max(mx, t);
      bytes += 88.0 * t;
    }
    if (mx <= 0) continue;
    TraceScope trace(GF2_TRACE_POST, b.count, bytes, s);
    hipLaunchKernelGGL(strassen_post_args_kernel, dim3(multi_x(mx, b.count), b.count), dim3(kThreads), 0, s, b);
    gf2_status r = hip_check(hipGetLastError(), "strassen_post_ops launch");
    if (r != GF2_OK) return r;
  }
  return GF2_OK;
}

gf2_status fill_zero_multi(const OView* dev_ops, int n, int64_t max_elems, hipStream_t s) {
  if (n <= 0 || max_elems <= 0) return GF2_OK;
  hipLaunchKernelGGL(fill_zero_multi_kernel, dim3(multi_x(max_elems, n), n), dim3(kThreads), 0, s, dev_ops);
  return hip_check(hipGetLastError(), "fill_zero_multi launch");
}

gf2_status strassen_pre_multi(const PreOp* dev_ops, int n, int64_t max_elems, hipStream_t s) {
  if (n <= 0 || max_elems <= 0) return GF2_OK;
  hipLaunchKernelGGL(strassen_pre_multi_kernel, dim3(multi_x(max_elems, n), n), dim3(kThreads), 0, s, dev_ops);
  return hip_check(hipGetLastError(), "strassen_pre_multi launch");
}

gf2_status strassen_post_multi(const PostOp* dev_ops, int n, int64_t max_elems, hipStream_t s) {
  if (n <= 0 || max_elems <= 0) return GF2_OK;
  hipLaunchKernelGGL(strassen_post_multi_kernel, dim3(multi_x(max_elems, n), n), dim3(kThreads), 0, s, dev_ops);
  return hip_check(hipGetLastError(), "strassen_post_multi launch");
}

}  // namespace gf2

namespace gf2 {
namespace {
// Timing operands: bit j of word w of the buffer is set with probability ``density``,
// from a hash of (seed, position); padding and stride gaps are ordinary bits here.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__global__ void fill_random_kernel(uint64_t* p, int64_t nwords, uint64_t seed, uint32_t thr, int dense) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t base = seed + (uint64_t)i * 0x9E3779B97F4A7C15ull;
    if (dense) {
      p[i] = mix64(base);
      continue;
    }
    uint64_t w = 0;
    for (int b = 0; b < 64; b += 2) {
      const uint64_t r = mix64(base + (uint64_t)b);
      w |= (uint64_t)((uint32_t)r < thr) << b;
      w |= (uint64_t)((uint32_t)(r >> 32) < thr) << (b + 1);
    }
    p[i] = w;
  }
}
}  // namespace

gf2_status fill_random(uint64_t* p, int64_t nwords, uint64_t seed, double density, hipStream_t s) {
  if (nwords <= 0) return GF2_OK;
  const int dense = density >= 0.5 - 1e-12 && density <= 0.5 + 1e-12;
  const double t = density <= 0 ? 0.0 : (density >= 1 ? 4294967295.0 : density * 4294967296.0);
  hipLaunchKernelGGL(fill_random_kernel, dim3(grid_for(nwords)), dim3(kThreads), 0, s, p, nwords, seed,
                     (uint32_t)t, dense);
  return hip_check(hipGetLastError(), "fill_random launch");
}

}  // namespace gf2
