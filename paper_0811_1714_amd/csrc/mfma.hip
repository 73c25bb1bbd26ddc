// Exact int8 matrix-core base case.  Over the integers, with A and B holding 0/1
// entries, (A B)[i][j] counts the t with A[i][t] = B[t][j] = 1; over GF(2) the
// product is that count mod 2 (the parity of Section 2.3's AND-and-accumulate).
// v_mfma_i32_32x32x32_i8 accumulates in int32 and bit 0 of the sum is the GF(2) result.
//
// B is first transposed (64 x 64 bit blocks) into Bt, k-word-major: Bt[w][j] holds bits
// 64w..64w+63 of column j.  Then A rows and Bt columns have k contiguous, and both are
// expanded the same way, in registers, from words staged through LDS.
//
// Expansion: for a nibble x, x * 0x204081 = x + (x << 7) + (x << 14) + (x << 21) puts bit
// b at positions b + 7j, all sixteen distinct (no carries), and bit 0 of byte b is bit b
// (position 8b, j = b); the other copies land on bits 1..7 of the bytes.  So byte b is odd
// exactly when bit b is set: byte b = bit b + 2 * (something).  A sum of products of such
// bytes (as signed or unsigned int8) has the parity of the sum of products of the bits,
// which is all the GF(2) result needs (int32 wrap-around would not change the parity
// either), so no mask is applied.
//
// Tile: 256 x 256 of C per workgroup of 8 waves; wave (wr, wc) owns rows 128*wr .. +128 and
// columns 64*wc .. +64 as 4 x 2 tiles of 32 x 32.  A stage is four k words: the workgroup
// copies 256 rows of A and 256 columns of Bt (32 B each) into LDS rows of 48 B (conflict-free
// ds_read_b64 for 16 consecutive rows), double-buffered, the next stage loaded into
// registers while the current one is multiplied.  The k slot of byte b in lane group g is
// 16g + b for both operands, so the pairing of A and B values does not depend on the
// order in which the hardware sums them.  Parities are packed into C words by a ballot.
#include <vector>

#include "gf2_internal.h"

namespace gf2 {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int TM = 4, TN = 2;              // 32x32 tiles per wave (rows, columns)
constexpr int WM = 2, WN = 4;              // waves per workgroup (rows, columns)
constexpr int NT = WM * WN * 64;           // 512 threads
constexpr int BMR = WM * TM * 32;          // 256 rows of C
constexpr int BNC = WN * TN * 32;          // 256 columns of C
constexpr int BNW = BNC / 64;              // 4 words
constexpr int KS = 4;                      // k words per stage
constexpr int RS = 12;                     // dwords per staged row: 8 data + 4 pad (48 B)
constexpr int STAGE = BMR * RS;            // dwords per operand per stage buffer

__device__ __forceinline__ int64_t imin64(int64_t a, int64_t b) { return a < b ? a : b; }

__device__ __forceinline__ int xcd_remap_mf(int i, int n) {
  const int per = n / 8, rem = n % 8;
  const int x = i % 8, idx = i / 8;
  return x < rem ? x * (per + 1) + idx : rem * (per + 1) + (x - rem) * per + idx;
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t mk_rsrc(const void* base, int64_t bytes) {
  const int nrec = bytes <= 0 ? 0 : (bytes >= 0x7fffffff ? 0x7fffffff : (int)bytes);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, nrec, 0x00020000);
}
__device__ __forceinline__ uint2 ld2(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

// 16 bits (starting at bit `sh` of x) -> 16 bytes whose parities are those bits.
__device__ __forceinline__ v4i expand16(uint32_t x, uint32_t sh) {
  v4i r;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    r[q] = (int)__umul24(__builtin_amdgcn_ubfe(x, sh + 4 * q, 4), 0x204081u);
  return r;
}

__device__ __forceinline__ void store_bits32(uint32_t* p, uint32_t v, int out) {
  if (out == OUT_STORE) *p = v;
  else if (out == OUT_XOR) *p ^= v;
  else if (v) atomicXor(p, v);
}

// d.B is Bt (k-word-major, d.ldb words between k words), d.k, d.n as for B.
__device__ void mfma_tile(const MulDesc& d, int tm, int tn, uint32_t* sA, uint32_t* sB) {
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int L = tid & 63;
  const int wr = w / WN, wc = w % WN;
  const int64_t row0 = (int64_t)tm * BMR, col0 = (int64_t)tn * BNC;   // tile origin (rows, columns)
  const int64_t Wn = words(d.n);
  const int kw = (int)words(d.k);
  const int nst = (kw + KS - 1) / KS;
  const int64_t ldt = d.ldb;                                          // Bt words per k word
  const int64_t cols = imin64(64 * Wn - col0, BNC);                   // Bt columns of this tile

  // Staging: thread t copies row (or column) t >> 1, k words 2(t & 1) and 2(t & 1) + 1.
  // A: one resource per wave (its 32 rows), so 32-bit offsets stay small.
  const int sr = tid >> 1, sh2 = tid & 1;
  const int64_t arow = row0 + 32 * w;
  const int rows_w = (int)imin64(d.m - arow, 32);
  const int lda_b = (int)(d.lda * 8);
  const __amdgpu_buffer_rsrc_t ra =
      mk_rsrc(d.A + arow * d.lda, rows_w > 0 ? (int64_t)(rows_w - 1) * lda_b + 8 * (int64_t)kw : 0);
  uint2 ga[2], gb[2];
  auto fetch = [&](int st) {
    const int kb = st * KS + 2 * sh2;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      ga[e] = ld2(ra, (sr - 32 * w) * lda_b + 8 * (kb + e));
      // Bt row kb + e (past k: zero), columns col0 .. col0 + cols.
      const bool in_k = kb + e < kw;
      const __amdgpu_buffer_rsrc_t rb = mk_rsrc(d.B + (int64_t)(in_k ? kb + e : 0) * ldt + col0, in_k ? 8 * cols : 0);
      gb[e] = ld2(rb, 8 * sr);
    }
  };
  auto stash = [&](int buf) {
    uint32_t* a = sA + buf * STAGE + sr * RS + 4 * sh2;
    uint32_t* b = sB + buf * STAGE + sr * RS + 4 * sh2;
    *reinterpret_cast<uint4*>(a) = make_uint4(ga[0].x, ga[0].y, ga[1].x, ga[1].y);
    *reinterpret_cast<uint4*>(b) = make_uint4(gb[0].x, gb[0].y, gb[1].x, gb[1].y);
  };

  v16i acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = v16i{0};

  if (nst > 0) {
    fetch(0);
    stash(0);
  }
  __syncthreads();
  const uint32_t gsh = 16u * (uint32_t)(L >> 5);       // this lane's 16 k values of a 32-k step
  for (int st = 0; st < nst; ++st) {
    if (st + 1 < nst) fetch(st + 1);
    const uint32_t* a = sA + (st & 1) * STAGE;
    const uint32_t* b = sB + (st & 1) * STAGE;
    const int ke = kw - st * KS < KS ? kw - st * KS : KS;               // k words in this stage
    for (int e = 0; e < ke; ++e) {
      uint2 aw[TM], bw[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) aw[i] = *reinterpret_cast<const uint2*>(a + (wr * TM * 32 + i * 32 + (L & 31)) * RS + 2 * e);
#pragma unroll
      for (int j = 0; j < TN; ++j) bw[j] = *reinterpret_cast<const uint2*>(b + (wc * TN * 32 + j * 32 + (L & 31)) * RS + 2 * e);
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        v4i af[TM], bf[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) af[i] = expand16(ks ? aw[i].y : aw[i].x, gsh);
#pragma unroll
        for (int j = 0; j < TN; ++j) bf[j] = expand16(ks ? bw[j].y : bw[j].x, gsh);
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af[i], bf[j], acc[i][j], 0, 0, 0);
      }
    }
    if (st + 1 < nst) stash((st + 1) & 1);
    __syncthreads();
  }

  // Parities -> bits.  Accumulator element e of lane L sits at row 8*(e/4) + 4*(L/32) + e%4,
  // column L%32 of its 32 x 32 tile; a ballot over the wave yields 32 columns of two rows.
  const int64_t n = d.n;
#pragma unroll
  for (int i = 0; i < TM; ++i) {
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int64_t colb = col0 + wc * TN * 32 + j * 32;                // first column of the tile
      const int64_t dcol = colb >> 5;                                   // dword index in a C row
      const int valid = (int)(n - colb < 0 ? 0 : (n - colb > 32 ? 32 : n - colb));
      const uint32_t vmask = valid >= 32 ? 0xffffffffu : ((1u << valid) - 1u);
      const bool in_words = dcol < 2 * Wn;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const uint64_t bal = __ballot(acc[i][j][e] & 1);
        const int64_t rbase = row0 + wr * TM * 32 + i * 32 + 8 * (e >> 2) + (e & 3);
        if ((L == 0 || L == 32) && in_words) {
          const int64_t r = rbase + 4 * (L >> 5);
          if (r < d.m) {
            const uint32_t bits = (L == 0 ? (uint32_t)bal : (uint32_t)(bal >> 32)) & vmask;
            store_bits32(reinterpret_cast<uint32_t*>(d.C + r * d.ldc) + dcol, bits, d.out);
          }
        }
      }
    }
  }
}

__global__ __launch_bounds__(NT) void mfma_group(GroupArgs g) {
  __shared__ __attribute__((aligned(16))) uint32_t sA[2 * STAGE];
  __shared__ __attribute__((aligned(16))) uint32_t sB[2 * STAGE];
  const int t = xcd_remap_mf(blockIdx.x, gridDim.x);
  int i = 0;
  while (i + 1 < g.count && g.tile_start[i + 1] <= t) ++i;
  const MulDesc& d = g.d[i];
  const int local = t - g.tile_start[i];
  const int tiles_m = (d.m + BMR - 1) / BMR;
  mfma_tile(d, local % tiles_m, local / tiles_m, sA, sB);
}

}  // namespace

int64_t mfma_tiles(const MulDesc& d) {
  return ((d.m + BMR - 1) / BMR) * ((words(d.n) + BNW - 1) / BNW);
}

gf2_status mfma_launch_group(const MulDesc* descs, int count, uint64_t* scratch, hipStream_t s) {
  // Transpose each product's B into its own scratch slice; the kernels read Bt.
  std::vector<MulDesc> bt(descs, descs + count);
  uint64_t* p = scratch;
  for (MulDesc& d : bt) {
    if (d.m <= 0 || d.n <= 0 || d.k <= 0) continue;
    gf2_status st = transpose_launch(d, p, s);
    if (st != GF2_OK) return st;
    d.B = p;
    d.ldb = 64 * words(d.n);
    p += transpose_words(d);
  }
  descs = bt.data();
  int i = 0;
  while (i < count) {
    GroupArgs g;
    g.count = 0;
    int64_t total = 0;
    double work = 0;
    for (; i < count && g.count < kMaxGroup; ++i) {
      const int64_t t = mfma_tiles(descs[i]);
      if (t == 0) continue;
      g.d[g.count] = descs[i];
      g.tile_start[g.count] = (int)total;
      ++g.count;
      total += t;
      work += (double)descs[i].m * descs[i].k * (double)descs[i].n;
      if (total > INT32_MAX) return set_error(GF2_ERR_UNSUPPORTED, "mfma: too many tiles in one launch");
    }
    if (g.count == 0) continue;
    g.tile_start[g.count] = (int)total;
    g.remap_n = (int)total;
    TraceScope trace(GF2_TRACE_MFMA, g.count, work, s);
    hipLaunchKernelGGL(mfma_group, dim3((unsigned)total), dim3(NT), 0, s, g);
    gf2_status st = hip_check(hipGetLastError(), "mfma_group launch");
    if (st != GF2_OK) return st;
  }
  return GF2_OK;
}

}  // namespace gf2
