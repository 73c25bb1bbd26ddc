// Popcount base case (Section 2.3): the dot product of row i of A with column j of B
// is the parity of the AND of the two, taken word by word with B stored transposed.
// Since parity is additive mod 2, the words are first combined by XOR and one
// popcount per (i, j) gives the bit.  The 64 parities of a wave (lanes = columns)
// are packed into one C word by a ballot: the "64 parities in parallel" of the paper.
//
// Bt is B transposed into k-word-major order: Bt[w*ldt + j] holds bits 64w..64w+63
// of column j, so that the lanes of a wave (consecutive j) read consecutive words.
#include "gf2_internal.h"

namespace gf2 {
namespace {

constexpr int CR = 16;   // rows of A per wave

// One wave transposes the 64 x 64 bit block (k words w, column word c) of B: lane t
// starts with row 64w+t; after six rounds that swap off-diagonal half blocks
// (32, 16, ..., 1) lane j holds column 64c+j.
__global__ __launch_bounds__(256) void transpose_kernel(const uint64_t* __restrict__ B, int64_t ldb, int64_t k,
                                                        int64_t Wn, int64_t Wk, uint64_t* __restrict__ Bt,
                                                        int64_t ldt) {
  const int64_t blk = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (blk >= Wk * Wn) return;
  const int lane = threadIdx.x & 63;
  const int64_t w = blk / Wn, c = blk % Wn;
  const int64_t row = w * 64 + lane;
  uint64_t x = row < k ? B[row * ldb + c] : 0ull;
  uint64_t m = 0x00000000FFFFFFFFull;
#pragma unroll
  for (int j = 32; j != 0; j >>= 1) {
    const uint64_t other = __shfl_xor(x, j);
    if ((lane & j) == 0) {
      const uint64_t t = ((x >> j) ^ other) & m;
      x ^= t << j;
    } else {
      const uint64_t t = ((other >> j) ^ x) & m;
      x ^= t;
    }
    m ^= m << (j >> 1);
  }
  Bt[w * ldt + c * 64 + lane] = x;
}

__device__ __forceinline__ void store_word(uint64_t* p, uint64_t v, int out) {
  if (out == OUT_STORE) *p = v;
  else if (out == OUT_XOR) *p ^= v;
  else if (v) atomicXor(reinterpret_cast<unsigned long long*>(p), (unsigned long long)v);
}

struct CubicArgs {
  MulDesc d;
  const uint64_t* Bt;
  int64_t ldt;
};

// Wave = (group of CR rows, one 64-column word).  Lane j accumulates, per row r,
// XOR over words w of (A[r][w] AND Bt[w][j]); parity via popcount; ballot packs
// the 64 columns into one word of C.
__global__ __launch_bounds__(256) void cubic_kernel(CubicArgs a) {
  const MulDesc& d = a.d;
  const int64_t Wn = words(d.n), Wk = words(d.k);
  const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t groups = (d.m + CR - 1) / CR;
  if (wave >= groups * Wn) return;
  const int lane = threadIdx.x & 63;
  const int64_t c = wave % Wn, r0 = (wave / Wn) * CR;
  const int rows = (int)((d.m - r0) < CR ? (d.m - r0) : CR);
  const uint64_t* bcol = a.Bt + c * 64 + lane;
  uint64_t acc[CR];
#pragma unroll
  for (int r = 0; r < CR; ++r) acc[r] = 0;
  const uint64_t* arow = d.A + r0 * d.lda;
  for (int64_t w = 0; w < Wk; ++w) {
    const uint64_t b = bcol[w * a.ldt];
#pragma unroll
    for (int r = 0; r < CR; ++r)
      if (r < rows) acc[r] ^= arow[r * d.lda + w] & b;
  }
  const uint64_t tail = (d.n & 63) && c == Wn - 1 ? ((1ull << (d.n & 63)) - 1) : ~0ull;
#pragma unroll
  for (int r = 0; r < CR; ++r) {
    const uint64_t bits = __ballot(__popcll(acc[r]) & 1) & tail;
    if (lane == 0 && r < rows) store_word(d.C + (r0 + r) * d.ldc + c, bits, d.out);
  }
}

}  // namespace

size_t cubic_scratch_words(const MulDesc& d) { return (size_t)words(d.k) * (size_t)(64 * words(d.n)); }

gf2_status transpose_launch(const MulDesc& d, uint64_t* bt, hipStream_t s) {
  const int64_t Wn = words(d.n), Wk = words(d.k);
  if (Wn == 0 || Wk == 0) return GF2_OK;
  const int64_t blocks = (Wk * Wn + 3) / 4;
  TraceScope tr(GF2_TRACE_CUBIC, 0, 16.0 * Wk * Wn * 64, s);   // transpose: bytes read + written
  hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)blocks), dim3(256), 0, s, d.B, d.ldb, (int64_t)d.k, Wn, Wk, bt,
                     64 * Wn);
  return hip_check(hipGetLastError(), "transpose launch");
}

gf2_status cubic_launch(const MulDesc& d, uint64_t* scratch, hipStream_t s) {
  const int64_t Wn = words(d.n), Wk = words(d.k);
  if (d.m == 0 || Wn == 0) return GF2_OK;
  const int64_t ldt = 64 * Wn;
  if (Wk > 0) {
    gf2_status st = transpose_launch(d, scratch, s);
    if (st != GF2_OK) return st;
  }
  CubicArgs a{d, scratch, ldt};
  const int64_t waves = ((d.m + CR - 1) / CR) * Wn;
  TraceScope tr(GF2_TRACE_CUBIC, 1, (double)d.m * d.n * (double)Wk, s);
  hipLaunchKernelGGL(cubic_kernel, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, a);
  return hip_check(hipGetLastError(), "cubic launch");
}

}  // namespace gf2
