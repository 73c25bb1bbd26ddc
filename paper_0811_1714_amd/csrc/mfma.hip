// Exact int8 matrix-core base case.  Over the integers, with A and B holding 0/1
// entries, (A B)[i][j] counts the t with A[i][t] = B[t][j] = 1; over GF(2) the
// product is that count mod 2 (the parity of Section 2.3's AND-and-accumulate).
// v_mfma_i32_32x32x32_i8 accumulates the exact count in int32 (it never exceeds
// k < 2^31, so no overflow), and bit 0 of the sum is the GF(2) result.
//
// Tile: 256 x 256 of C per workgroup of 8 waves; wave (wr, wc) owns rows
// 128*wr .. +128 and columns 64*wc .. +64 as 4 x 2 tiles of 32 x 32.  Per 64-bit
// step of k, A's rows are expanded nibble by nibble into 0/1 bytes in LDS (row-major,
// k contiguous), and B's columns are gathered bit by bit from staged B words into
// 0/1 bytes (column-major, k contiguous), the operand layout the matrix core wants.
// The k slot of byte b in lane group g is 16*g + b for both operands, so the pairing
// of A and B values is the same whatever order the hardware sums them in.
// Parities are packed back into C words with a wave ballot.
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
constexpr int ES = 20;                     // dwords per expanded row (64 bytes + pad: conflict-free b128)

// Nibble -> four 0/1 bytes (bit b of x to byte b): the shifts 0, 7, 14, 21 do not overlap.
__device__ __forceinline__ uint32_t nib_bytes(uint32_t x) { return __umul24(x, 0x204081u) & 0x01010101u; }

__device__ __forceinline__ int xcd_remap_mf(int i, int n) {
  const int per = n / 8, rem = n % 8;
  const int x = i % 8, idx = i / 8;
  return x < rem ? x * (per + 1) + idx : rem * (per + 1) + (x - rem) * per + idx;
}

__device__ __forceinline__ void store_bits32(uint32_t* p, uint32_t v, int out) {
  if (out == OUT_STORE) *p = v;
  else if (out == OUT_XOR) *p ^= v;
  else if (v) atomicXor(p, v);
}

__device__ void mfma_tile(const MulDesc& d, int tm, int tn, uint32_t* Ae, uint32_t* Be, uint64_t* Bs) {
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int L = tid & 63;
  const int wr = w / WN, wc = w % WN;
  const int64_t row0 = (int64_t)tm * BMR, cw0 = (int64_t)tn * BNW;   // tile origin (rows, words)
  const int64_t Wn = words(d.n);
  const int kw = (int)words(d.k);
  const uint64_t ktail = (d.k & 63) ? ((1ull << (d.k & 63)) - 1) : ~0ull;

  v16i acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = v16i{0};

  for (int kb = 0; kb < kw; ++kb) {
    // Stage the 64 x 256 block of B bits (64 rows of k, 4 words each).
    for (int idx = tid; idx < 64 * BNW; idx += NT) {
      const int t = idx / BNW, c = idx % BNW;
      const int64_t kr = (int64_t)kb * 64 + t, wcol = cw0 + c;
      Bs[idx] = (kr < d.k && wcol < Wn) ? d.B[kr * d.ldb + wcol] : 0ull;
    }
    // Expand A: row r, 16-bit quarter q of this k word -> 4 dwords of 0/1 bytes.
    for (int idx = tid; idx < BMR * 4; idx += NT) {
      const int r = idx >> 2, q = idx & 3;
      uint64_t a = 0;
      if (row0 + r < d.m) {
        a = d.A[(row0 + r) * d.lda + kb];
        if (kb == kw - 1) a &= ktail;
      }
      const uint32_t h = (uint32_t)(a >> (16 * q)) & 0xffffu;
      *reinterpret_cast<uint4*>(Ae + r * ES + 4 * q) =
          make_uint4(nib_bytes(h & 15), nib_bytes((h >> 4) & 15), nib_bytes((h >> 8) & 15), nib_bytes(h >> 12));
    }
    __syncthreads();
    // Expand B: column c, k rows 16q .. 16q+15 -> 4 dwords of 0/1 bytes (k contiguous).
    for (int idx = tid; idx < BNC * 4; idx += NT) {
      const int c = idx >> 2, q = idx & 3;
      const uint32_t* half = reinterpret_cast<const uint32_t*>(Bs) + ((c >> 6) * 2 + ((c >> 5) & 1));
      const int sh = c & 31;
      uint32_t v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        uint32_t x = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int t = 16 * q + 4 * e + b;
          x |= ((half[t * 2 * BNW] >> sh) & 1u) << (8 * b);
        }
        v[e] = x;
      }
      *reinterpret_cast<uint4*>(Be + c * ES + 4 * q) = make_uint4(v[0], v[1], v[2], v[3]);
    }
    __syncthreads();
    // Two 32-deep matrix-core steps.
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const int dw = 8 * ks + 4 * (L >> 5);       // dwords of this lane's 16 k values
      v4i af[TM], bf[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const uint4 u = *reinterpret_cast<const uint4*>(Ae + (wr * TM * 32 + i * 32 + (L & 31)) * ES + dw);
        af[i] = v4i{(int)u.x, (int)u.y, (int)u.z, (int)u.w};
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const uint4 u = *reinterpret_cast<const uint4*>(Be + (wc * TN * 32 + j * 32 + (L & 31)) * ES + dw);
        bf[j] = v4i{(int)u.x, (int)u.y, (int)u.z, (int)u.w};
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }

  // Parities -> bits.  Accumulator element e of lane L sits at row 8*(e/4) + 4*(L/32) + e%4,
  // column L%32 of its 32 x 32 tile; a ballot over the wave yields 32 columns of two rows.
  const int64_t n = d.n;
#pragma unroll
  for (int i = 0; i < TM; ++i) {
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int64_t colb = (cw0 * 64) + wc * TN * 32 + j * 32;        // first column of the tile
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
  __shared__ __attribute__((aligned(16))) uint32_t Ae[BMR * ES];
  __shared__ __attribute__((aligned(16))) uint32_t Be[BNC * ES];
  __shared__ uint64_t Bs[64 * BNW];
  const int t = xcd_remap_mf(blockIdx.x, gridDim.x);
  int i = 0;
  while (i + 1 < g.count && g.tile_start[i + 1] <= t) ++i;
  const MulDesc& d = g.d[i];
  const int local = t - g.tile_start[i];
  const int tiles_m = (d.m + BMR - 1) / BMR;
  mfma_tile(d, local % tiles_m, local / tiles_m, Ae, Be, Bs);
}

}  // namespace

int64_t mfma_tiles(const MulDesc& d) {
  return ((d.m + BMR - 1) / BMR) * ((words(d.n) + BNW - 1) / BNW);
}

gf2_status mfma_launch_group(const MulDesc* descs, int count, hipStream_t s) {
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
