// Popcount base case (Section 2.3): the dot product of row i of A with column j of B
// is the parity of the AND of the two, taken word by word with B stored transposed.
// Since parity is additive mod 2, the words are first combined by XOR and one
// popcount per (i, j) gives the bit.  The 64 parities of a wave (lanes = columns)
// are packed into one C word by a ballot: the "64 parities in parallel" of the paper.
//
// Bt is B transposed into k-word-major order: Bt[w*ldt + j] holds bits 64w..64w+63
// of column j, so that the lanes of a wave (consecutive j) read consecutive words.
#include <algorithm>

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

// Narrow B (n <= 8 columns: matrix-vector products and their few-column relatives).  Each
// wave owns whole rows of A and streams them once: lane l takes words l, l + 64, ... of the
// row (512 contiguous bytes per load instruction, eight loads in flight per lane), ANDs each
// with the same word of every column of B, and counts bits; the row's parity per column is
// the parity of the sum over the wave, one ballot each.  The N columns of B (transposed,
// zero past k and padded with zeros to a whole number of batches) sit in LDS for the whole
// block, so A is the only stream from HBM.  Words past the row read as zero through the
// buffer range check.
constexpr int kNarrowBatch = 8;                           // loads in flight per lane
constexpr int64_t kNarrowStep = 64 * kNarrowBatch;        // words of a row per batch

__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void* base, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

// Columns 0..nc-1 of B (n <= 8, one word per row) as bit vectors: word w of column j,
// at cols[j*Wp + w], holds rows 64w..64w+63; zero past k, up to Wp words.  One wave per
// word: lane l reads row 64w + l, one ballot per column.
__global__ __launch_bounds__(256) void narrow_columns_kernel(const uint64_t* __restrict__ B, int64_t ldb, int64_t k,
                                                             int nc, int64_t Wp, uint64_t* __restrict__ cols) {
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= Wp) return;
  const int lane = threadIdx.x & 63;
  const int64_t row = w * 64 + lane;
  const uint64_t x = row < k ? B[row * ldb] : 0ull;
  for (int j = 0; j < nc; ++j) {
    const uint64_t v = __ballot((x >> j) & 1);
    if (lane == j) cols[j * Wp + w] = v;
  }
}

template <int N>
__global__ __launch_bounds__(256) void narrow_kernel(CubicArgs a) {
  extern __shared__ uint64_t cols[];                      // N x Wp words, column j at j*Wp
  const MulDesc& d = a.d;
  const int64_t Wk = words(d.k);
  const int64_t Wp = (Wk + kNarrowStep - 1) / kNarrowStep * kNarrowStep;
  for (int64_t x = threadIdx.x; x < N * Wp; x += 256) cols[x] = a.Bt[x];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const uint64_t tail = (1ull << d.n) - 1;                // n <= 8
  for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < d.m; i += (int64_t)gridDim.x * 4) {
    const __amdgpu_buffer_rsrc_t ra = row_rsrc(d.A + i * d.lda, Wk * 8);
    uint32_t cnt[N];
#pragma unroll
    for (int j = 0; j < N; ++j) cnt[j] = 0;
    for (int64_t w0 = lane; w0 < Wp; w0 += kNarrowStep) {
      uint64_t x[kNarrowBatch];
#pragma unroll
      for (int u = 0; u < kNarrowBatch; ++u) {
        const uint2 v = __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(ra, (int)((w0 + 64 * u) * 8), 0, 0));
        x[u] = (uint64_t)v.x | ((uint64_t)v.y << 32);
      }
#pragma unroll
      for (int u = 0; u < kNarrowBatch; ++u)
#pragma unroll
        for (int j = 0; j < N; ++j) cnt[j] += (uint32_t)__popcll(x[u] & cols[j * Wp + w0 + 64 * u]);
    }
    uint64_t bits = 0;
#pragma unroll
    for (int j = 0; j < N; ++j) bits |= (uint64_t)(__popcll(__ballot(cnt[j] & 1)) & 1) << j;
    if (lane == 0) store_word(d.C + i * d.ldc, bits & tail, d.out);
  }
}

constexpr int kNarrowCols = 8;
constexpr int64_t kNarrowLdsBytes = 65536;

int narrow_width(int n) { return n <= 1 ? 1 : n <= 2 ? 2 : n <= 4 ? 4 : 8; }
int64_t narrow_padded_words(int64_t k) { return (words(k) + kNarrowStep - 1) / kNarrowStep * kNarrowStep; }

}  // namespace

bool cubic_narrow_shape(int64_t k, int64_t n) {
  return n >= 1 && n <= kNarrowCols && k >= 1 && (int64_t)narrow_width((int)n) * narrow_padded_words(k) * 8 <= kNarrowLdsBytes;
}

bool cubic_narrow(const MulDesc& d) { return cubic_narrow_shape(d.k, d.n); }

size_t transpose_words(const MulDesc& d) { return (size_t)words(d.k) * (size_t)(64 * words(d.n)); }

size_t cubic_scratch_words(const MulDesc& d) {
  if (cubic_narrow(d)) return (size_t)narrow_width(d.n) * (size_t)narrow_padded_words(d.k);
  return transpose_words(d);
}

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
  if (cubic_narrow(d)) {
    const int nw = narrow_width(d.n);
    const int64_t Wp = narrow_padded_words(d.k);
    const size_t lds = (size_t)nw * (size_t)Wp * 8;
    {
      TraceScope tc(GF2_TRACE_CUBIC, 0, 16.0 * (double)Wp * 64, s);
      hipLaunchKernelGGL(narrow_columns_kernel, dim3((unsigned)((Wp + 3) / 4)), dim3(256), 0, s, d.B, d.ldb,
                         (int64_t)d.k, nw, Wp, scratch);
      gf2_status st = hip_check(hipGetLastError(), "narrow columns launch");
      if (st != GF2_OK) return st;
    }
    CubicArgs a{d, scratch, Wp};
    const int64_t blocks = std::min<int64_t>((d.m + 3) / 4, 2048);
    TraceScope tr(GF2_TRACE_CUBIC, 2, (double)d.m * d.n * (double)Wk, s);
    switch (nw) {
      case 1: hipLaunchKernelGGL(narrow_kernel<1>, dim3((unsigned)blocks), dim3(256), lds, s, a); break;
      case 2: hipLaunchKernelGGL(narrow_kernel<2>, dim3((unsigned)blocks), dim3(256), lds, s, a); break;
      case 4: hipLaunchKernelGGL(narrow_kernel<4>, dim3((unsigned)blocks), dim3(256), lds, s, a); break;
      default: hipLaunchKernelGGL(narrow_kernel<8>, dim3((unsigned)blocks), dim3(256), lds, s, a); break;
    }
    return hip_check(hipGetLastError(), "narrow launch");
  }
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
