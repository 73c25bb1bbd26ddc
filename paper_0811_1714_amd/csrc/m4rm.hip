// M4RM base case for gfx950: the Method of the Four Russians (Section 3 of the
// paper, Algorithms 1-3) with the Gray-code table build of Section 3.1.
//
// Tile families (t tables of 8-bit indices per barrier phase, Algorithm 3): t = 1 on
// 2048-column tiles, t = 2 on 1024, t = 4 on 512 (the large-product kernel), t = 8 on
// 256 and t = 32 on one-word tiles.  Each keeps its tables in one 64 KiB LDS buffer per
// phase, double buffered.  The t = 1 form is described first:
//
// Mapping onto a CDNA4 compute unit:
//  * A workgroup owns a C tile of BM = WAVES*RW rows by 2048 columns (32 words);
//    the tile lives in VGPRs for the whole k loop and is written once (the row
//    blocking of Algorithm 2, with registers in the role of the cache).
//  * k is consumed in stripes of KB = 8 rows of B.  For each stripe the
//    workgroup builds the table T[x] = XOR of rows kp+b of B with bit b of x set
//    (all 2^8 combinations, 256 B per entry) in LDS, walking a Gray code so that
//    every entry after the first costs one row addition.  Tables are double
//    buffered: stripe p+1 is built while stripe p is looked up, one barrier per
//    stripe.
//  * Lookup ("ReadBits" + "AddRowFromTable"): byte p%4 of an A dword is the
//    8-bit index of row r for stripe p (column j at bit j&63, so the index is
//    LSB-first: bit b <-> row kp+b).  One v_perm builds the LDS address
//    (index in byte 1, lane offset in byte 0, buffer in byte 2); one ds_read_b128
//    serves four rows per wave instruction (16 lanes x 16 B = one 256 B entry
//    per row), the pattern that measured fastest on gfx950 LDS.
#include <algorithm>
#include <type_traits>

#include "gf2_internal.h"

namespace gf2 {
namespace {

constexpr int KB = 8;                       // table width (kappa)
constexpr int TILE_WORDS = 32;              // 2048 columns per tile
constexpr int ENTRY_BYTES = TILE_WORDS * 8; // 256 B per table entry
constexpr int TABLE_BYTES = (1 << KB) * ENTRY_BYTES;  // 64 KiB

// Integer clamps (the generic min/max overloads of device code may go through double).
__device__ __forceinline__ int64_t imin64(int64_t a, int64_t b) { return a < b ? a : b; }

__device__ __forceinline__ uint4 xor4(uint4 a, uint4 b) {
  return make_uint4(a.x ^ b.x, a.y ^ b.y, a.z ^ b.z, a.w ^ b.w);
}

// Raw buffer resource over [base, base + bytes): loads at offsets >= bytes return 0
// (the hardware range check), which is how rows past k, rows past m and words past
// the end of a row are read as zero without branches.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, int64_t bytes) {
  const int nrec = bytes <= 0 ? 0 : (bytes >= 0x7fffffff ? 0x7fffffff : (int)bytes);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, nrec, 0x00020000);
}
// The same for a range known to fit 31 bits (negative means empty), in 32-bit scalar arithmetic.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc32(const void* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes > 0 ? bytes : 0, 0x00020000);
}
__device__ __forceinline__ uint2 bload2(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ uint32_t bload1(__amdgpu_buffer_rsrc_t r, int off) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
}

// C is global memory: said explicitly, so that tiles compiled as functions of their own (the
// persistent kernel's) store with global rather than flat instructions.
using gword = __attribute__((address_space(1))) uint64_t;

__device__ __forceinline__ void store_word(uint64_t* cp, uint64_t v, int out) {
  gword* gp = (gword*)cp;
  if (out == OUT_STORE) {
    *gp = v;
  } else if (out == OUT_XOR) {
    *gp ^= v;
  } else {
    if (v) atomicXor(reinterpret_cast<unsigned long long*>(cp), (unsigned long long)v);
  }
}

// Workgroup-to-tile map: the hardware deals workgroups to the 8 XCDs round-robin;
// give each XCD a contiguous range of logical tiles so that neighbouring tiles
// (same B column panel) share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int i, int n) {
  const int per = n / 8, rem = n % 8;
  const int x = i % 8, idx = i / 8;
  return x < rem ? x * (per + 1) + idx : rem * (per + 1) + (x - rem) * per + idx;
}

template <int WAVES, int RW>
struct Tile {
  static constexpr int S = RW / 4;          // row slots per lane (4 rows per wave instruction)
  static constexpr int BM = WAVES * RW;
  static constexpr int WB = WAVES == 16 ? 4 : WAVES == 8 ? 3 : WAVES == 4 ? 2 : 1;
  static_assert((1 << WB) == WAVES, "WAVES must be 2, 4, 8 or 16");
  static_assert(RW % 8 == 0, "RW must be a multiple of 8");
};

// Rows of B for one stripe, one dword per lane: lane j holds columns 32j..32j+31 of
// the tile for each of the KAPPA rows (rows past k and words past the row read as zero).
template <int KAPPA = KB>
struct StripeRows {
  uint32_t r[KAPPA];
};

// log2 of a workgroup's wave count (2, 4, 8 or 16 waves).
template <int WAVES>
constexpr int wave_bits() { return WAVES == 16 ? 4 : WAVES == 8 ? 3 : WAVES == 4 ? 2 : 1; }

// Byte offsets of a lane's KAPPA rows of B from the start of a phase of ``phase_rows`` rows,
// the lane's first row at ``boff``.  A wave needs the rows that select its fixed high index
// bits (b >= HIB) only where that bit of w is set; the others are pointed one phase further
// on, past the end of the phase's buffer range, so they load as zero.  The loads then need
// no branches, which keeps the compiler's count of loads in flight exact (a branch around a
// load makes it wait for loads it does not need).
template <int HIB, int KAPPA>
__device__ __forceinline__ void row_offsets(int (&o)[KAPPA], int boff, int ldb_b, int phase_rows, int w) {
#pragma unroll
  for (int b = 0; b < KAPPA; ++b) {
    const bool need = b < HIB || ((w >> (b - HIB)) & 1);
    o[b] = boff + (b + (need ? 0 : phase_rows)) * ldb_b;
  }
}

// Index bytes per row of A for table width KAPPA: KAPPA = 8 reads A itself (byte j of a
// row = bits 8j..8j+7); a narrower table reads A's index expansion (byte j = bits
// KAPPA*j .. KAPPA*j+KAPPA-1, see expand_indices), so every lookup takes one byte either way.
template <int KAPPA>
__device__ __forceinline__ int index_bytes(int k) { return (k + KAPPA - 1) / KAPPA; }

template <int WAVES>
__device__ __forceinline__ void load_stripe(StripeRows<>& sr, const uint64_t* pb, int64_t ldb, int rows,
                                            int64_t row_bytes, int w, int lane) {
  constexpr int HIB = KB - wave_bits<WAVES>();  // walked rows
#pragma unroll
  for (int b = 0; b < KB; ++b) {
    // Rows selecting the wave's fixed high bits are only needed when that bit of w is set;
    // the others get an empty range (they load as zero, with no branch around the load).
    const bool need = b < HIB || ((w >> (b - HIB)) & 1);
    const __amdgpu_buffer_rsrc_t r = make_rsrc(pb + b * ldb, (b < rows && need) ? row_bytes : 0);
    sr.r[b] = bload1(r, lane * 4);
  }
}

// Build this wave's share of one stripe's table into LDS buffer ``buf``: the entries
// x = (w << HIB) | g(i), i < 2^HIB, g the binary reflected Gray code, HIB = KAPPA minus the
// wave-count bits.  Bit b of x selects B row kp+b, so T[x] = XOR of the selected rows;
// consecutive Gray codes differ in exactly bit ctz(i), hence each further entry costs one
// row addition (Section 3.1).  One wave instruction writes one whole 256 B entry (lane j =
// dword j); a table of width KAPPA has 2^KAPPA entries.
template <int WAVES, int KAPPA = KB>
__device__ __forceinline__ void build_table(char* tab, int buf, int w, int lane, const StripeRows<KAPPA>& sr) {
  constexpr int HIB = KAPPA - wave_bits<WAVES>();
  static_assert(HIB >= 0, "every wave must own at least one table entry");
  uint32_t v = 0;
#pragma unroll
  for (int b = HIB; b < KAPPA; ++b) v ^= sr.r[b];    // zero where w's bit is clear
  char* dst = tab + ((uint32_t)buf << 16) + lane * 4;
  const uint32_t base = (uint32_t)w << HIB;
  *reinterpret_cast<uint32_t*>(dst + base * ENTRY_BYTES) = v;
#pragma unroll
  for (int i = 1; i < (1 << HIB); ++i) {
    v ^= sr.r[__builtin_ctz(i)];
    *reinterpret_cast<uint32_t*>(dst + (base | (uint32_t)(i ^ (i >> 1))) * ENTRY_BYTES) = v;
  }
}

// One C tile of BM rows x 2048 columns.  EDGE = the tile reaches past the last row or
// word of C, or its last word has padding bits: stores are guarded and masked.
template <int WAVES, int RW, bool EDGE>
__device__ __forceinline__ void m4rm_tile(const MulDesc& d, int tm, int tn, char* tab) {
  using T = Tile<WAVES, RW>;
  constexpr int S = T::S;
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int L = tid & 63, q = L >> 4, l16 = L & 15;
  const int64_t Wn = words(d.n);
  const int lw = 2 * l16;                               // this lane's word offset inside the tile
  const int64_t c0 = (int64_t)tn * TILE_WORDS;          // tile's first word column (uniform)
  const int64_t Wt = Wn - c0;                           // valid words from the tile start
  const int64_t row0 = (int64_t)tm * T::BM + (int64_t)w * RW;   // first row of this wave (uniform)
  const int rows_here = (int)imin64(d.m - row0, RW);
  const int nstripes = (d.k + KB - 1) / KB;
  const int kdw = (d.k + 31) >> 5;                      // A dwords per row that hold bits < k
  const uint32_t lanebase = (uint32_t)l16 * 16u;

  // A indices: dword g of a row holds the 8-bit indices of stripes 4g..4g+3.  Each lane
  // keeps the dwords of its own row slots for the current group and prefetches the next
  // group's; offsets past the wave's last existing row read as zero.
  const int lda_b = (int)(d.lda * 8);
  const __amdgpu_buffer_rsrc_t ra =
      make_rsrc(d.A + row0 * d.lda, rows_here > 0 ? (int64_t)(rows_here - 1) * lda_b + 4 * kdw : 0);

  uint4 acc[S];
#pragma unroll
  for (int s = 0; s < S; ++s) acc[s] = make_uint4(0, 0, 0, 0);
  // Two register sets of A dwords swap roles every group (current / prefetched), so
  // the prefetch needs no copies and is waited for only when it is used.
  uint32_t ax[S], ay[S];
  auto load_a = [&](int g, uint32_t (&dst)[S]) {
#pragma unroll
    for (int s = 0; s < S; ++s) dst[s] = bload1(ra, (4 * s + q) * lda_b + 4 * g);
  };

  // B rows of stripe p+1 are loaded before the lookups of stripe p, so their latency
  // is hidden behind the lookups; the table is built from them afterwards.
  StripeRows<> sr;
  auto fetch = [&](int p) {
    const int64_t kp = (int64_t)p * KB;
    load_stripe<WAVES>(sr, d.B + kp * d.ldb + c0, d.ldb, (int)imin64(d.k - kp, KB), 8 * Wt, w, L);
  };
  if (nstripes > 0) {
    load_a(0, ax);
    fetch(0);
    build_table<WAVES>(tab, 0, w, L, sr);
  }
  __syncthreads();

  // One stripe: lookups of stripe p in table buffer p&1 with byte U of the A dwords,
  // then the table of stripe p+1 into the other buffer.
  auto stripe = [&](int p, auto U, const uint32_t (&aw)[S]) {
    if (p + 1 < nstripes) fetch(p + 1);
    const uint32_t lb = lanebase | ((uint32_t)(p & 1) << 16);
    constexpr uint32_t sel = 0x0c020400u + ((uint32_t)decltype(U)::value << 8);  // byte0 <- lb, byte1 <- A byte U, byte2 <- lb
    constexpr int INFL = WAVES >= 16 ? 2 : 4;          // lookups in flight per wave
#pragma unroll
    for (int s0 = 0; s0 < S; s0 += INFL) {
#pragma unroll
      for (int s = s0; s < s0 + INFL && s < S; ++s) {
        const uint32_t addr = __builtin_amdgcn_perm(aw[s], lb, sel);
        acc[s] = xor4(acc[s], *reinterpret_cast<const uint4*>(tab + addr));
      }
      // Register fence: the XORs of this group complete here, so at most INFL
      // lookups are in flight and none is held across the table build.
#pragma unroll
      for (int s = s0; s < s0 + INFL && s < S; ++s)
        asm volatile("" : "+v"(acc[s].x), "+v"(acc[s].y), "+v"(acc[s].z), "+v"(acc[s].w));
    }
    if (p + 1 < nstripes) build_table<WAVES>(tab, (p & 1) ^ 1, w, L, sr);
    __syncthreads();
  };
  // A group: four stripes sharing one set of A dwords; the next group's set is loaded first.
  auto group = [&](int g, const uint32_t (&cur)[S], uint32_t (&nxt)[S]) {
    const int p0 = 4 * g;
    if (p0 + 4 < nstripes) load_a(g + 1, nxt);
    stripe(p0, std::integral_constant<int, 0>{}, cur);
    if (p0 + 1 < nstripes) stripe(p0 + 1, std::integral_constant<int, 1>{}, cur);
    if (p0 + 2 < nstripes) stripe(p0 + 2, std::integral_constant<int, 2>{}, cur);
    if (p0 + 3 < nstripes) stripe(p0 + 3, std::integral_constant<int, 3>{}, cur);
  };
  const int ngroups = (nstripes + 3) >> 2;
  for (int g = 0; g < ngroups; g += 2) {
    group(g, ax, ay);
    if (g + 1 < ngroups) group(g + 1, ay, ax);
  }

  // Store: rows < m, words < Wn; padding bits of the last word are cleared.
  const uint64_t tail = (d.n & 63) ? ((1ull << (d.n & 63)) - 1) : ~0ull;
  const uint64_t m0 = (EDGE && lw == Wt - 1) ? tail : ~0ull;
  const uint64_t m1 = (EDGE && lw + 1 == Wt - 1) ? tail : ~0ull;
  uint64_t* pc = d.C + row0 * d.ldc + c0 + lw;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int rr = 4 * s + q;
    if (!EDGE || rr < rows_here) {
      uint64_t* cp = pc + (int64_t)rr * d.ldc;
      const uint64_t w0 = ((uint64_t)acc[s].x | ((uint64_t)acc[s].y << 32)) & m0;
      const uint64_t w1 = ((uint64_t)acc[s].z | ((uint64_t)acc[s].w << 32)) & m1;
      if (!EDGE || lw < Wt) store_word(cp, w0, d.out);
      if (!EDGE || lw + 1 < Wt) store_word(cp + 1, w1, d.out);
    }
  }
}

template <int WAVES, int RW>
__device__ __forceinline__ void m4rm_tile_any(const MulDesc& d, int tm, int tn, char* tab) {
  using T = Tile<WAVES, RW>;
  const int64_t Wn = words(d.n);
  const bool edge = (int64_t)(tm + 1) * T::BM > d.m || (int64_t)(tn + 1) * TILE_WORDS > Wn ||
                    ((d.n & 63) != 0 && (int64_t)(tn + 1) * TILE_WORDS == Wn);
  if (edge) m4rm_tile<WAVES, RW, true>(d, tm, tn, tab);
  else m4rm_tile<WAVES, RW, false>(d, tm, tn, tab);
}

// Up to kMaxGroup products in one launch, descriptors passed by value (no device
// staging, so the launch can be captured into a graph as is).  Workgroup b belongs to
// the product i with tile_start[i] <= b < tile_start[i+1].
// ---------------------------------------------------------------------------
// Two tables per phase (Algorithm 3 with t = 2).  The tile is 1024 columns wide,
// so the pair of 8-bit tables of a 16-row phase of B fits one 64 KiB buffer,
// interleaved: entry x of table h (h = 0, 1) at x*256 + h*128, column dword j at
// +4j.  One ds_write_b32 wave instruction writes entry x of both tables (lanes
// 0-31 walk the Gray code over rows kp..kp+7, lanes 32-63 over kp+8..kp+15), and
// one v_bitop3 folds both lookups of a row into its accumulator
// ("AddTwoRowsFromTable").  Eight rows per lookup instruction (8 lanes x 16 B per
// 128 B half-entry).  Halving the tile width doubles the rows that share each table.
// Rows of odd 8-lane groups look up the two tables in the opposite order, so every
// 16 lanes of a lookup instruction cover both halves of the 64 LDS banks (table 0 in
// banks 0-31, table 1 in banks 32-63) instead of contending for one half.
constexpr int T2_WORDS = 16;                // 1024 columns per tile

// B rows are loaded D phases ahead of the build that uses them (a ring of D register sets,
// indexed by the phase modulo D, which the unrolled code knows at compile time).  Measured in
// the persistent batch kernel: two phases ahead helps the four-table tiles of up to 1024 rows
// (2-6% per product), while the two-table tiles, and any tile at four phases ahead, lose more
// to the extra registers (saved and restored around each tile) than the shorter wait gains.
template <int S, int TABLES>
constexpr int prefetch_depth() { return TABLES == 4 && S <= 4 ? 2 : 1; }

template <int WAVES, int S, int KAPPA = KB>
struct Tile2 {
  static constexpr int RW = 8 * S;          // rows per wave: eight per lookup instruction
  static constexpr int BM = WAVES * RW;
  static constexpr int HIB = KAPPA - wave_bits<WAVES>();
  static constexpr int PR = 2 * KAPPA;      // rows of B per phase
  static constexpr int D = prefetch_depth<S, 2>();   // B prefetch depth in phases (divides 8)
};

__device__ __forceinline__ uint4 xor3v(uint4 a, uint4 b, uint4 c) {
  return make_uint4(__builtin_amdgcn_bitop3_b32(a.x, b.x, c.x, 0x96), __builtin_amdgcn_bitop3_b32(a.y, b.y, c.y, 0x96),
                    __builtin_amdgcn_bitop3_b32(a.z, b.z, c.z, 0x96), __builtin_amdgcn_bitop3_b32(a.w, b.w, c.w, 0x96));
}

template <int WAVES, int S, int INFL, int KAPPA, bool EDGE>
__device__ __forceinline__ void m4rm2_tile(const MulDesc& d, int tm, int tn, char* tab) {
  using T = Tile2<WAVES, S, KAPPA>;
  constexpr int D = T::D;
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int L = tid & 63, g8 = L >> 3, l8 = L & 7;
  const int64_t Wn = words(d.n);
  const int lw = 2 * l8;                                // lane's word offset inside the tile
  const int64_t c0 = (int64_t)tn * T2_WORDS;            // tile's first word column (uniform)
  const int64_t Wt = Wn - c0;                           // valid words from the tile start
  const int64_t row0 = (int64_t)tm * T::BM + (int64_t)w * T::RW;
  const int rows_here = (int)imin64(d.m - row0, T::RW);
  const int nphases = (d.k + T::PR - 1) / T::PR;
  const int kdw = (index_bytes<KAPPA>(d.k) + 3) >> 2;   // A dwords per row that hold indices
  const int lda_b = (int)(d.lda * 8), ldb_b = (int)(d.ldb * 8);
  // A: dword gd of a row holds the indices of phases 2gd (bytes 0, 1) and 2gd+1 (bytes 2, 3).
  const __amdgpu_buffer_rsrc_t ra =
      make_rsrc(d.A + row0 * d.lda, rows_here > 0 ? (int64_t)(rows_here - 1) * lda_b + 4 * kdw : 0);
  // Odd 8-lane groups read table 1 first: their first lookup takes the table-1 index into
  // the table-1 half, their second the table-0 index into the table-0 half.
  const uint32_t hsw = (uint32_t)g8 & 1u;
  const uint32_t lb0 = hsw * 128u + (uint32_t)l8 * 16u, lb1 = (hsw ^ 1u) * 128u + (uint32_t)l8 * 16u;
  // v_perm selectors of the two lookups of phase half U (index bytes 2U and 2U+1 of the A
  // dword): byte0 <- low address byte, byte1 <- index byte, byte2 <- buffer bit, byte3 <- 0.
  const uint32_t asel00 = 0x0c020400u + (hsw << 8), asel01 = 0x0c020400u + ((1u - hsw) << 8);
  const uint32_t asel10 = asel00 + 0x200u, asel11 = asel01 + 0x200u;
  // Tiles of more than eight slots per lane (no registers to spare) swap the A byte pairs
  // of odd groups in place instead and load one dword per group.
  const uint32_t swp = hsw ? 0x02030001u : 0x03020100u;
  // B: lane L builds column dword L&31 of table L>>5, i.e. rows kp + 8*(L>>5) + b.
  const int boff = (L >> 5) * KAPPA * ldb_b + (L & 31) * 4;
  int bo[KAPPA];
  row_offsets<T::HIB, KAPPA>(bo, boff, ldb_b, T::PR, w);

  uint4 acc[S];
#pragma unroll
  for (int s = 0; s < S; ++s) acc[s] = make_uint4(0, 0, 0, 0);
  // A: dword gd of a row serves phases 2gd and 2gd+1.  Every eight phases, lane (row slot r,
  // chunk lane l) loads dword 4c + (l & 3) of its row for each slot s (both quads of a row's
  // eight lanes hold the same four dwords), so one load covers 8 rows x 16 contiguous bytes;
  // group gd = 4c + jj takes dword jj from its quad with a quad broadcast (DPP).  Chunk c + 1
  // is loaded at the start of chunk c, eight phases ahead of its use.
  uint32_t ax[S], ay[S];
  auto load_chunk = [&](int c, uint32_t (&dst)[S]) {
#pragma unroll
    for (int s = 0; s < S; ++s) dst[s] = bload1(ra, (8 * s + g8) * lda_b + 16 * c + 4 * (l8 & 3));
  };
  StripeRows<KAPPA> ring[D];
  auto fetch = [&](int p, StripeRows<KAPPA>& sr) {
    const int64_t kp = (int64_t)p * T::PR;
    const int rows = (int)imin64(d.k - kp, T::PR);
    const __amdgpu_buffer_rsrc_t rb = make_rsrc(d.B + kp * d.ldb + c0, (int64_t)(rows - 1) * ldb_b + 8 * Wt);
#pragma unroll
    for (int b = 0; b < KAPPA; ++b) sr.r[b] = bload1(rb, bo[b]);
  };
  constexpr bool kChunked = S <= 8;
  auto load_a = [&](int gd, uint32_t (&dst)[S]) {
#pragma unroll
    for (int s = 0; s < S; ++s) dst[s] = bload1(ra, (8 * s + g8) * lda_b + 4 * gd);
  };
  if (nphases > 0) {
    if constexpr (kChunked) load_chunk(0, ax);
    else load_a(0, ax);
#pragma unroll
    for (int i = 0; i < D; ++i) fetch(i, ring[i]);        // phases 0 .. D-1
    build_table<WAVES, KAPPA>(tab, 0, w, L, ring[0]);
  }
  __syncthreads();

  // Lookups of phase p with the A dword of each slot given by ``dword(s)``; U = p & 1 picks
  // the index bytes.  The next phase's B rows (and, at the start of a chunk, the next chunk
  // of A) are loaded unconditionally: past the end the B range is empty and the A offsets
  // stay inside the tile's rows (or past the range, reading zero), and the data is never
  // used.  Keeping branches away from the loads lets the compiler wait for exactly the loads
  // each step needs.
  auto lookups = [&](int p, uint32_t s0sel, uint32_t s1sel, auto dword, const StripeRows<KAPPA>& next_rows) {
    const uint32_t buf = (uint32_t)(p & 1) << 16;
#pragma unroll
    for (int s0 = 0; s0 < S; s0 += INFL) {
#pragma unroll
      for (int s = s0; s < s0 + INFL && s < S; ++s) {
        const uint32_t aw = dword(s);
        const uint4 t0 = *reinterpret_cast<const uint4*>(tab + __builtin_amdgcn_perm(aw, lb0 | buf, s0sel));
        const uint4 t1 = *reinterpret_cast<const uint4*>(tab + __builtin_amdgcn_perm(aw, lb1 | buf, s1sel));
        acc[s] = xor3v(acc[s], t0, t1);
      }
#pragma unroll
      for (int s = s0; s < s0 + INFL && s < S; ++s)
        asm volatile("" : "+v"(acc[s].x), "+v"(acc[s].y), "+v"(acc[s].z), "+v"(acc[s].w));
    }
    if (p + 1 < nphases) build_table<WAVES, KAPPA>(tab, (p & 1) ^ 1, w, L, next_rows);
    __syncthreads();
  };
  // Phase p = 8c + 2jj + U of chunk c (jj, U compile-time): its B rows leave ring slot p mod D,
  // which then receives phase p + D's.
  auto phase = [&](int p, auto JJ, auto U, const uint32_t (&cur)[S], uint32_t (&nxt)[S]) {
    constexpr int jj = decltype(JJ)::value, u = decltype(U)::value, slot = (2 * jj + u) % D;
    fetch(p + D, ring[slot]);
    if constexpr (jj == 0 && u == 0) load_chunk((p >> 3) + 1, nxt);
    lookups(p, u ? asel10 : asel00, u ? asel11 : asel01,
            [&](int s) { return (uint32_t)__builtin_amdgcn_mov_dpp((int)cur[s], jj * 0x55, 0xf, 0xf, true); },
            ring[(slot + 1) % D]);
  };
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  using I3 = std::integral_constant<int, 3>;
  auto chunk = [&](int c, uint32_t (&cur)[S], uint32_t (&nxt)[S]) {
    const int p = 8 * c;
    phase(p, I0{}, I0{}, cur, nxt);
    phase(p + 1, I0{}, I1{}, cur, nxt);
    phase(p + 2, I1{}, I0{}, cur, nxt);
    phase(p + 3, I1{}, I1{}, cur, nxt);
    phase(p + 4, I2{}, I0{}, cur, nxt);
    phase(p + 5, I2{}, I1{}, cur, nxt);
    phase(p + 6, I3{}, I0{}, cur, nxt);
    phase(p + 7, I3{}, I1{}, cur, nxt);
  };
  // The one to seven phases of a last, partial chunk: the dword comes from the quad's lane
  // jj through ds_bpermute (jj known only at run time); speed does not matter here.
  // Unrolled by D, so that each phase's ring slot is known at compile time.
  auto part = [&](int c, const uint32_t (&cur)[S]) {
    for (int p0 = 8 * c; p0 < nphases; p0 += D) {
#pragma unroll
      for (int i = 0; i < D; ++i) {
        const int p = p0 + i;
        if (p < nphases) {
          fetch(p + D, ring[i]);
          const int jj = (p >> 1) & 3, u = p & 1;
          const int src = ((L & ~3) | jj) * 4;
          lookups(p, u ? asel10 : asel00, u ? asel11 : asel01,
                  [&](int s) { return (uint32_t)__builtin_amdgcn_ds_bpermute(src, (int)cur[s]); }, ring[(i + 1) % D]);
        }
      }
    }
  };
  if constexpr (kChunked) {
    // Whole chunks with A alternating between ax and ay, then the partial chunk.
    const int full = nphases >> 3;
    int c = 0;
    for (; c + 1 < full; c += 2) {
      chunk(c, ax, ay);
      chunk(c + 1, ay, ax);
    }
    if (c < full) {
      chunk(c, ax, ay);
      part(c + 1, ay);
    } else {
      part(c, ax);
    }
  } else {
    // One A dword per group (two phases), loaded a group ahead; byte pairs swapped in place.
    constexpr uint32_t sel00 = 0x0c020400u, sel01 = 0x0c020500u, sel10 = 0x0c020600u, sel11 = 0x0c020700u;
    auto group = [&](int gd, uint32_t (&cur)[S], uint32_t (&nxt)[S]) {
      const int p0 = 2 * gd;
      load_a(gd + 1, nxt);
#pragma unroll
      for (int s = 0; s < S; ++s) cur[s] = __builtin_amdgcn_perm(cur[s], cur[s], swp);
      static_assert(D == 1, "tiles of more than eight slots fetch one phase ahead");
      fetch(p0 + 1, ring[0]);
      lookups(p0, sel00, sel01, [&](int s) { return cur[s]; }, ring[0]);
      if (p0 + 1 < nphases) {
        fetch(p0 + 2, ring[0]);
        lookups(p0 + 1, sel10, sel11, [&](int s) { return cur[s]; }, ring[0]);
      }
    };
    const int ngroups = (nphases + 1) >> 1;
    for (int gd = 0; gd < ngroups; gd += 2) {
      group(gd, ax, ay);
      if (gd + 1 < ngroups) group(gd + 1, ay, ax);
    }
  }

  const uint64_t tail = (d.n & 63) ? ((1ull << (d.n & 63)) - 1) : ~0ull;
  const uint64_t m0 = (EDGE && lw == Wt - 1) ? tail : ~0ull;
  const uint64_t m1 = (EDGE && lw + 1 == Wt - 1) ? tail : ~0ull;
  uint64_t* pc = d.C + row0 * d.ldc + c0 + lw;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int rr = 8 * s + g8;
    if (!EDGE || rr < rows_here) {
      uint64_t* cp = pc + (int64_t)rr * d.ldc;
      const uint64_t w0 = ((uint64_t)acc[s].x | ((uint64_t)acc[s].y << 32)) & m0;
      const uint64_t w1 = ((uint64_t)acc[s].z | ((uint64_t)acc[s].w << 32)) & m1;
      if (!EDGE || lw < Wt) store_word(cp, w0, d.out);
      if (!EDGE || lw + 1 < Wt) store_word(cp + 1, w1, d.out);
    }
  }
}

template <int WAVES, int S, int INFL, int KAPPA>
__device__ __forceinline__ void m4rm2_tile_any(const MulDesc& d, int tm, int tn, char* tab) {
  using T = Tile2<WAVES, S, KAPPA>;
  const int64_t Wn = words(d.n);
  const bool edge = (int64_t)(tm + 1) * T::BM > d.m || (int64_t)(tn + 1) * T2_WORDS > Wn ||
                    ((d.n & 63) != 0 && (int64_t)(tn + 1) * T2_WORDS == Wn);
  if (edge) m4rm2_tile<WAVES, S, INFL, KAPPA, true>(d, tm, tn, tab);
  else m4rm2_tile<WAVES, S, INFL, KAPPA, false>(d, tm, tn, tab);
}

// ---------------------------------------------------------------------------
// Eight tables per phase (Algorithm 3 with t = 8) for narrow products.  The tile is 256
// columns (4 words) wide, so the eight 8-bit tables of a 64-row phase of B fit one 64 KiB
// buffer, interleaved: entry x of table h at x*256 + h*32.  The build is the same Gray
// walk as above: one ds_write_b32 wave instruction writes entry x of all eight tables
// (lane L: table L>>3, column dword L&7).  Lookups: two lanes per row (16 B each), so one
// ds_read_b128 serves 32 rows.  In lookup instruction h, row r reads table h ^ (r & 7):
// every 16 lanes then touch eight different tables, i.e. all 64 LDS banks.  Each row's A
// qword (its eight indices for the phase) is byte-permuted once so that instruction h
// finds row r's index for table h ^ (r & 7) in byte h.  A is loaded in chunks of two
// phases: lane (row, half j) loads the row's qword of phase 2c + j, so one load instruction
// covers 32 rows x 16 contiguous bytes, and phase 2c + j takes its qword from the row's
// half-j lane with a quad broadcast (DPP).  Loading 8 bytes per row per phase instead, one
// instruction touched 32 cache lines for 256 bytes of indices, four times the lines per
// index byte of the four-table tile.
constexpr int T8_WORDS = 4;                 // 256 columns per tile

template <int WAVES, int S, int KAPPA = KB>
struct Tile8 {
  static constexpr int RW = 32 * S;         // rows per wave: 32 per lookup instruction
  static constexpr int BM = WAVES * RW;
  static constexpr int HIB = KAPPA - wave_bits<WAVES>();
  static constexpr int PR = 8 * KAPPA;      // rows of B per phase
  // B rows are loaded DA phases ahead, DA = 2 on the short tiles: a ring of DA sets of B rows
  // indexed by the phase modulo 4.  A chunks (two phases each) are loaded one chunk ahead.
  static constexpr int DA = S <= 2 ? 2 : 1;
};

template <int WAVES, int S, int KAPPA, bool EDGE>
__device__ __forceinline__ void m4rm8_tile(const MulDesc& d, int tm, int tn, char* tab) {
  using T = Tile8<WAVES, S, KAPPA>;
  constexpr int DA = T::DA;
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int L = tid & 63, r32 = L >> 1, half = L & 1;
  const int64_t Wn = words(d.n);
  const int lw = 2 * half;                              // lane's word offset inside the tile
  const int64_t c0 = (int64_t)tn * T8_WORDS;            // tile's first word column (uniform)
  const int64_t Wt = Wn - c0;                           // valid words from the tile start
  const int64_t row0 = (int64_t)tm * T::BM + (int64_t)w * T::RW;
  const int rows_here = (int)imin64(d.m - row0, T::RW);
  const int nphases = (d.k + T::PR - 1) / T::PR;
  const int kq = (index_bytes<KAPPA>(d.k) + 7) >> 3;    // A words per row that hold indices
  const int lda_b = (int)(d.lda * 8), ldb_b = (int)(d.ldb * 8);
  const __amdgpu_buffer_rsrc_t ra =
      make_rsrc(d.A + row0 * d.lda, rows_here > 0 ? (int64_t)(rows_here - 1) * lda_b + 8 * kq : 0);
  // Lookup address, low byte: table (h ^ rr)*32 + half*16 = cb ^ (h*32), rr = r & 7.
  const uint32_t rr = (uint32_t)r32 & 7u;
  const uint32_t cb = (rr << 5) | ((uint32_t)half << 4);
  // Byte permutation of the A qword {hi:lo}: result byte b = source byte b ^ rr.
  uint32_t sel_lo = 0, sel_hi = 0;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    sel_lo |= ((uint32_t)b ^ rr) << (8 * b);
    sel_hi |= ((uint32_t)(4 + b) ^ rr) << (8 * b);
  }
  // B: lane L builds column dword L&7 of table L>>3, i.e. rows kp + 8*(L>>3) + b.
  const int boff = (L >> 3) * KAPPA * ldb_b + (L & 7) * 4;
  int bo[KAPPA];
  row_offsets<T::HIB, KAPPA>(bo, boff, ldb_b, T::PR, w);

  uint4 acc[S];
#pragma unroll
  for (int s = 0; s < S; ++s) acc[s] = make_uint4(0, 0, 0, 0);
  uint2 ach[2][S];                                      // A chunk c in set c & 1
  auto load_chunk = [&](int c, uint2 (&dst)[S]) {
#pragma unroll
    for (int s = 0; s < S; ++s) dst[s] = bload2(ra, (32 * s + r32) * lda_b + 16 * c + 8 * half);
  };
  StripeRows<KAPPA> ring[DA];
  auto fetch = [&](int p, StripeRows<KAPPA>& sr) {
    const int64_t kp = (int64_t)p * T::PR;
    const int rows = (int)imin64(d.k - kp, T::PR);
    const __amdgpu_buffer_rsrc_t rb = make_rsrc(d.B + kp * d.ldb + c0, (int64_t)(rows - 1) * ldb_b + 8 * Wt);
#pragma unroll
    for (int b = 0; b < KAPPA; ++b) sr.r[b] = bload1(rb, bo[b]);
  };
  if (nphases > 0) {
    load_chunk(0, ach[0]);
#pragma unroll
    for (int i = 0; i < DA; ++i) fetch(i, ring[i]);       // phases 0 .. DA-1
    build_table<WAVES, KAPPA>(tab, 0, w, L, ring[0]);
  }
  __syncthreads();

  // The next loads are issued unconditionally (past the end they load zeros or unused
  // stride-gap words, with no branch), and a chunk's byte permutation is pinned after the
  // barrier that ends the previous phase (an empty asm on each qword): hoisted above it, it
  // would wait there for loads that have only just been issued.
  auto phase = [&](int p, auto I) {
    constexpr int i = decltype(I)::value;                 // p mod 4
    constexpr int j = i & 1, cs = i >> 1;                 // phase 2c + j of chunk c, in set cs
    constexpr int dpp = j ? 0xf5 : 0xa0;                  // quad lanes {1,1,3,3} or {0,0,2,2}
    uint2 (&cur)[S] = ach[cs];
    fetch(p + DA, ring[i % DA]);
    if constexpr (j == 0) {
      load_chunk((p >> 1) + 1, ach[cs ^ 1]);
#pragma unroll
      for (int s = 0; s < S; ++s) {
        asm volatile("" : "+v"(cur[s].x), "+v"(cur[s].y));
        const uint32_t lo = __builtin_amdgcn_perm(cur[s].y, cur[s].x, sel_lo);
        const uint32_t hi = __builtin_amdgcn_perm(cur[s].y, cur[s].x, sel_hi);
        cur[s] = make_uint2(lo, hi);
      }
    }
    const uint32_t lb = cb | ((uint32_t)(p & 1) << 16);
    // byte0 <- lb ^ table offset, byte1 <- index byte h (of lo or hi), byte2 <- buffer bit
    constexpr uint32_t base_sel = 0x0c020400u;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      // The row's permuted qword for this phase, from its half-j lane.
      const uint32_t qlo = (uint32_t)__builtin_amdgcn_mov_dpp((int)cur[s].x, dpp, 0xf, 0xf, true);
      const uint32_t qhi = (uint32_t)__builtin_amdgcn_mov_dpp((int)cur[s].y, dpp, 0xf, 0xf, true);
#pragma unroll
      for (int h = 0; h < 8; h += 2) {
        const uint32_t l0 = lb ^ ((uint32_t)h << 5), l1 = lb ^ ((uint32_t)(h + 1) << 5);
        const uint32_t q = h < 4 ? qlo : qhi;
        const uint32_t a0 = __builtin_amdgcn_perm(q, l0, base_sel + ((uint32_t)(h & 3) << 8));
        const uint32_t a1 = __builtin_amdgcn_perm(q, l1, base_sel + ((uint32_t)((h + 1) & 3) << 8));
        const uint4 t0 = *reinterpret_cast<const uint4*>(tab + a0);
        const uint4 t1 = *reinterpret_cast<const uint4*>(tab + a1);
        acc[s] = xor3v(acc[s], t0, t1);
      }
      asm volatile("" : "+v"(acc[s].x), "+v"(acc[s].y), "+v"(acc[s].z), "+v"(acc[s].w));
    }
    if (p + 1 < nphases) build_table<WAVES, KAPPA>(tab, (p & 1) ^ 1, w, L, ring[(i + 1) % DA]);
    __syncthreads();
  };
  constexpr std::integral_constant<int, 0> I0{};
  constexpr std::integral_constant<int, 1> I1{};
  constexpr std::integral_constant<int, 2> I2{};
  constexpr std::integral_constant<int, 3> I3{};
  int p = 0;
  for (; p + 3 < nphases; p += 4) {
    phase(p, I0);
    phase(p + 1, I1);
    phase(p + 2, I2);
    phase(p + 3, I3);
  }
  if (p < nphases) phase(p, I0);
  if (p + 1 < nphases) phase(p + 1, I1);
  if (p + 2 < nphases) phase(p + 2, I2);

  const uint64_t tail = (d.n & 63) ? ((1ull << (d.n & 63)) - 1) : ~0ull;
  const uint64_t m0 = (EDGE && lw == Wt - 1) ? tail : ~0ull;
  const uint64_t m1 = (EDGE && lw + 1 == Wt - 1) ? tail : ~0ull;
  uint64_t* pc = d.C + row0 * d.ldc + c0 + lw;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int rrow = 32 * s + r32;
    if (!EDGE || rrow < rows_here) {
      uint64_t* cp = pc + (int64_t)rrow * d.ldc;
      const uint64_t w0 = ((uint64_t)acc[s].x | ((uint64_t)acc[s].y << 32)) & m0;
      const uint64_t w1 = ((uint64_t)acc[s].z | ((uint64_t)acc[s].w << 32)) & m1;
      if (!EDGE || lw < Wt) store_word(cp, w0, d.out);
      if (!EDGE || lw + 1 < Wt) store_word(cp + 1, w1, d.out);
    }
  }
}

template <int WAVES, int S, int KAPPA>
__device__ __forceinline__ void m4rm8_tile_any(const MulDesc& d, int tm, int tn, char* tab) {
  using T = Tile8<WAVES, S, KAPPA>;
  const int64_t Wn = words(d.n);
  const bool edge = (int64_t)(tm + 1) * T::BM > d.m || (int64_t)(tn + 1) * T8_WORDS > Wn ||
                    ((d.n & 63) != 0 && (int64_t)(tn + 1) * T8_WORDS == Wn);
  if (edge) m4rm8_tile<WAVES, S, KAPPA, true>(d, tm, tn, tab);
  else m4rm8_tile<WAVES, S, KAPPA, false>(d, tm, tn, tab);
}

// ---------------------------------------------------------------------------
// Four tables per phase (Algorithm 3 with t = 4) on 512-column (8-word) tiles: the four
// 8-bit tables of a 32-row phase of B fill one 64 KiB buffer, interleaved: entry x of
// table h at x*256 + h*64.  Per phase and per row this reads as many LDS bytes as the
// two-table tile (four 64 B half-rows instead of two 128 B ones) and builds a table of
// the same size, but a phase covers twice the rows of B and a tile holds twice the rows
// in the same registers (a lane's 16 B accumulator covers a quarter of a 512-bit row):
// half the table build per product bit, and half the barriers and B fetches per row of B.
// Build: the Gray walk above; lane L builds column dword L&15 of table L>>4.  Lookups:
// four lanes per row (16 B each), so one ds_read_b128 serves 16 rows.  In lookup
// instruction h, row r reads table h ^ (r & 3): the four rows of every 16-lane group hit
// four different tables, i.e. all 64 banks.  The address is one v_perm of the row's A dword
// (its four indices for the phase) with a per-lane selector that picks index byte h ^ (r & 3).
constexpr int T4_WORDS = 8;                 // 512 columns per tile

template <int WAVES, int S, int KAPPA = KB>
struct Tile4 {
  static constexpr int RW = 16 * S;         // rows per wave: 16 per lookup instruction
  static constexpr int BM = WAVES * RW;
  static constexpr int HIB = KAPPA - wave_bits<WAVES>();
  static constexpr int PR = 4 * KAPPA;      // rows of B per phase
  static constexpr int D = prefetch_depth<S, 4>();   // B prefetch depth in phases (divides 4)
};

template <int WAVES, int S, int KAPPA, bool EDGE>
__device__ __forceinline__ void m4rm4_tile(const MulDesc& d, int tm, int tn, char* tab) {
  using T = Tile4<WAVES, S, KAPPA>;
  constexpr int D = T::D;
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int L = tid & 63, r16 = L >> 2, qtr = L & 3;
  const int64_t Wn = words(d.n);
  const int lw = 2 * qtr;                               // lane's word offset inside the tile
  const int64_t c0 = (int64_t)tn * T4_WORDS;            // tile's first word column (uniform)
  const int64_t Wt = Wn - c0;                           // valid words from the tile start
  const int64_t row0 = (int64_t)tm * T::BM + (int64_t)w * T::RW;
  const int rows_here = (int)imin64(d.m - row0, T::RW);
  const int nphases = (d.k + T::PR - 1) / T::PR;
  const int kdw = (index_bytes<KAPPA>(d.k) + 3) >> 2;   // A dwords per row that hold indices
  const int lda_b = (int)(d.lda * 8), ldb_b = (int)(d.ldb * 8);
  const __amdgpu_buffer_rsrc_t ra =
      make_rsrc(d.A + row0 * d.lda, rows_here > 0 ? (int64_t)(rows_here - 1) * lda_b + 4 * kdw : 0);
  // Lookup address, low byte: table (h ^ rr)*64 + qtr*16 = cb ^ (h*64), rr = r & 3.
  const uint32_t rr = (uint32_t)r16 & 3u;
  const uint32_t cb = (rr << 6) | ((uint32_t)qtr << 4);
  // v_perm selectors of lookup instruction h: byte0 <- low address byte, byte1 <- the row's
  // index for table h ^ rr (byte h ^ rr of its A dword), byte2 <- buffer bit, byte3 <- 0.
  uint32_t asel[4];
#pragma unroll
  for (int h = 0; h < 4; ++h) asel[h] = 0x0c020400u + ((((uint32_t)h ^ rr)) << 8);
  // B: lane L builds column dword L&15 of table L>>4, i.e. rows kp + 8*(L>>4) + b, read at
  // offset boff from a buffer resource per b that starts at row kp + b.  Its range ends with
  // the phase's last row (rows at or past k read as zero), and is empty for a row that
  // selects one of the wave's fixed high index bits where that bit of w is clear (such a
  // row is not needed, and must read as zero).  One offset register serves all eight loads.
  const int boff = (L >> 4) * KAPPA * ldb_b + (L & 15) * 4;

  uint4 acc[S];
#pragma unroll
  for (int s = 0; s < S; ++s) acc[s] = make_uint4(0, 0, 0, 0);
  // A: every four phases, lane (row slot r, quarter q) loads dword 4c + q of its row for each
  // slot s, so one load instruction covers 16 rows x 16 contiguous bytes (four phases of
  // indices) instead of 16 rows x 4 bytes; phase 4c + j then takes dword j from the row's
  // quarter-j lane with a quad broadcast (DPP).  Chunk c + 1 is loaded at the start of
  // chunk c, four phases ahead of its use.
  uint32_t ax[S], ay[S];
  auto load_chunk = [&](int c, uint32_t (&dst)[S]) {
#pragma unroll
    for (int s = 0; s < S; ++s) dst[s] = bload1(ra, (16 * s + r16) * lda_b + 16 * c + 4 * qtr);
  };
  StripeRows<KAPPA> ring[D];
  // Ranges fit 31 bits: at most 31 rows of at most 2^24 bytes plus one row's valid bytes.
  const int wt_b = 8 * (int)Wt;
  // Phases are fetched in order, so the row pointer and the rows left advance by one phase
  // per call (no 64-bit multiply per phase).
  const char* bnext = reinterpret_cast<const char*>(d.B + c0);
  const int64_t bstep = (int64_t)T::PR * ldb_b;
  int64_t kleft = d.k;
  auto fetch = [&](StripeRows<KAPPA>& sr) {
    const int rows = (int)imin64(kleft, T::PR);           // > -PR * D even past the last phase
    const int last = (rows - 1) * ldb_b + wt_b;           // range from the phase's first row
    const char* rowp = bnext;                             // row kp + b, and its range
    int left = last;
#pragma unroll
    for (int b = 0; b < KAPPA; ++b) {
      const bool need = b < T::HIB || ((w >> (b - T::HIB)) & 1);
      sr.r[b] = bload1(make_rsrc32(rowp, need ? left : 0), boff);
      rowp += ldb_b;
      left -= ldb_b;
    }
    bnext += bstep;
    kleft -= T::PR;
  };
  if (nphases > 0) {
    load_chunk(0, ax);
#pragma unroll
    for (int i = 0; i < D; ++i) fetch(ring[i]);           // phases 0 .. D-1
    build_table<WAVES, KAPPA>(tab, 0, w, L, ring[0]);
  }
  __syncthreads();

  // Phase p = 4c + J of chunk c.  The B rows of phase p + D (into the ring slot phase p's rows
  // have just left) and, at J = 0, the next chunk of A are loaded unconditionally: past the end
  // the B range is empty and the A offsets stay inside the tile's rows (or past the range,
  // reading zero), and what they bring is never used.  Keeping branches away from the loads
  // lets the compiler wait for exactly the loads each step needs; B is issued first so the
  // table build waits for it alone.
  auto phase = [&](int p, auto J, uint32_t (&cur)[S], uint32_t (&nxt)[S]) {
    constexpr int j = decltype(J)::value;
    fetch(ring[j % D]);
    if constexpr (j == 0) load_chunk((p >> 2) + 1, nxt);
    const uint32_t lb = cb | ((uint32_t)(p & 1) << 16);
    const uint32_t l0 = lb, l1 = lb ^ 64u, l2 = lb ^ 128u, l3 = lb ^ 192u;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      // The row's four indices for this phase, then its four lookups (one per table).
      const uint32_t aw = (uint32_t)__builtin_amdgcn_mov_dpp((int)cur[s], j * 0x55, 0xf, 0xf, true);
      const uint4 t0 = *reinterpret_cast<const uint4*>(tab + __builtin_amdgcn_perm(aw, l0, asel[0]));
      const uint4 t1 = *reinterpret_cast<const uint4*>(tab + __builtin_amdgcn_perm(aw, l1, asel[1]));
      const uint4 t2 = *reinterpret_cast<const uint4*>(tab + __builtin_amdgcn_perm(aw, l2, asel[2]));
      const uint4 t3 = *reinterpret_cast<const uint4*>(tab + __builtin_amdgcn_perm(aw, l3, asel[3]));
      acc[s] = xor3v(xor3v(acc[s], t0, t1), t2, t3);
      asm volatile("" : "+v"(acc[s].x), "+v"(acc[s].y), "+v"(acc[s].z), "+v"(acc[s].w));
    }
    // Lookups run at a raised wave priority and the table build at the normal one, so waves
    // still looking up are issued ahead of waves already building (about 1% at 32768^3).
    __builtin_amdgcn_s_setprio(0);
    if (p + 1 < nphases) build_table<WAVES, KAPPA>(tab, (p & 1) ^ 1, w, L, ring[(j + 1) % D]);
    __syncthreads();
    __builtin_amdgcn_s_setprio(2);
  };
  constexpr std::integral_constant<int, 0> J0{};
  constexpr std::integral_constant<int, 1> J1{};
  constexpr std::integral_constant<int, 2> J2{};
  constexpr std::integral_constant<int, 3> J3{};
  auto chunk = [&](int c, uint32_t (&cur)[S], uint32_t (&nxt)[S]) {
    phase(4 * c, J0, cur, nxt);
    phase(4 * c + 1, J1, cur, nxt);
    phase(4 * c + 2, J2, cur, nxt);
    phase(4 * c + 3, J3, cur, nxt);
  };
  // The one to three phases of a last, partial chunk.
  auto part = [&](int c, uint32_t (&cur)[S], uint32_t (&nxt)[S]) {
    const int rem = nphases - 4 * c;
    if (rem > 0) phase(4 * c, J0, cur, nxt);
    if (rem > 1) phase(4 * c + 1, J1, cur, nxt);
    if (rem > 2) phase(4 * c + 2, J2, cur, nxt);
  };
  // Whole chunks with A alternating between ax and ay, then the partial chunk.
  const int full = nphases >> 2;
  int c = 0;
  for (; c + 1 < full; c += 2) {
    chunk(c, ax, ay);
    chunk(c + 1, ay, ax);
  }
  if (c < full) {
    chunk(c, ax, ay);
    part(c + 1, ay, ax);
  } else {
    part(c, ax, ay);
  }

  const uint64_t tail = (d.n & 63) ? ((1ull << (d.n & 63)) - 1) : ~0ull;
  const uint64_t m0 = (EDGE && lw == Wt - 1) ? tail : ~0ull;
  const uint64_t m1 = (EDGE && lw + 1 == Wt - 1) ? tail : ~0ull;
  uint64_t* pc = d.C + row0 * d.ldc + c0 + lw;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int rrow = 16 * s + r16;
    if (!EDGE || rrow < rows_here) {
      uint64_t* cp = pc + (int64_t)rrow * d.ldc;
      const uint64_t w0 = ((uint64_t)acc[s].x | ((uint64_t)acc[s].y << 32)) & m0;
      const uint64_t w1 = ((uint64_t)acc[s].z | ((uint64_t)acc[s].w << 32)) & m1;
      if (!EDGE || lw < Wt) store_word(cp, w0, d.out);
      if (!EDGE || lw + 1 < Wt) store_word(cp + 1, w1, d.out);
    }
  }
}

template <int WAVES, int S, int KAPPA>
__device__ __forceinline__ void m4rm4_tile_any(const MulDesc& d, int tm, int tn, char* tab) {
  using T = Tile4<WAVES, S, KAPPA>;
  const int64_t Wn = words(d.n);
  const bool edge = (int64_t)(tm + 1) * T::BM > d.m || (int64_t)(tn + 1) * T4_WORDS > Wn ||
                    ((d.n & 63) != 0 && (int64_t)(tn + 1) * T4_WORDS == Wn);
  if (edge) m4rm4_tile<WAVES, S, KAPPA, true>(d, tm, tn, tab);
  else m4rm4_tile<WAVES, S, KAPPA, false>(d, tm, tn, tab);
}

// ---------------------------------------------------------------------------
// One-word tiles (n <= 64: matrix-vector and narrow products), 32 tables per phase
// (Algorithm 3 with t = 32): 256 rows of B per phase, table entries of one 64-bit word.
// The tables are interleaved by LDS bank: entry x of table j at x*256 + j*8, so table j
// lives in bank pair j.  Four lanes share a row: lane quarter q loads the row's 8 index
// bytes of tables 8q..8q+7 for the phase (so one load instruction covers 16 rows x 32
// contiguous bytes) and looks those tables up; at step s the lane of row slot r reads
// table 8q + (s ^ (r & 7)), so the 32 lanes of an LDS pass (8 rows x 4 quarters) read
// 32 distinct bank pairs whatever their indices.  The 8 index bytes are permuted once
// per phase (byte b moves to b ^ (r & 7)) so that step s finds its index in byte s.
// The four quarters' partial sums are combined by XOR across lanes at the end.
// Build: thread (wave w, half h) holds the eight B rows of table j = lane & 31 and walks
// the Gray code over the low three index bits of entries (2w + h) << 3 | g.
constexpr int P32 = 32 * KB;                // rows of B per phase

template <int WAVES, int RPT>
struct Tile32 {
  static_assert(WAVES == 16, "the build maps 16 waves x 2 halves onto 32 high-bit groups");
  static constexpr int NT = WAVES * 64;
  static constexpr int RW = 16 * RPT;       // rows per wave: 16 per slot (4 lanes each)
  static constexpr int BM = WAVES * RW;
};

template <int WAVES, int RPT, bool EDGE>
__device__ __forceinline__ void m4rm32_tile(const MulDesc& d, int tm, int tn, char* tab) {
  using T = Tile32<WAVES, RPT>;
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int L = tid & 63;
  const uint32_t lr = (uint32_t)L & 31u;               // build: table of this lane
  const int q = L & 3, r16 = L >> 2;                    // lookup: quarter and row slot
  const uint32_t rx = (uint32_t)r16 & 7u;               // table rotation of this row slot
  const int64_t row0 = (int64_t)tm * T::BM + (int64_t)w * T::RW;
  const int rows_here = (int)imin64(d.m - row0, T::RW);
  const int nphases = (d.k + P32 - 1) / P32;
  const int kq = (d.k + 63) >> 6;                       // A words per row that hold bits < k
  const int lda_b = (int)(d.lda * 8), ldb_b = (int)(d.ldb * 8);
  const __amdgpu_buffer_rsrc_t ra =
      make_rsrc(d.A + row0 * d.lda, rows_here > 0 ? (int64_t)(rows_here - 1) * lda_b + 8 * kq : 0);
  // Byte permutation of the quarter's 8 index bytes {hi:lo}: result byte b = source b ^ rx.
  uint32_t sel_lo = 0, sel_hi = 0;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    sel_lo |= ((uint32_t)b ^ rx) << (8 * b);
    sel_hi |= ((uint32_t)(4 + b) ^ rx) << (8 * b);
  }

  uint2 acc[RPT], ax[RPT], ay[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) acc[i] = make_uint2(0, 0);
  auto load_a = [&](int p, uint2 (&dst)[RPT]) {
#pragma unroll
    for (int i = 0; i < RPT; ++i) dst[i] = bload2(ra, (16 * i + r16) * lda_b + 32 * p + 8 * q);
  };
  // B rows of table j = lane & 31 for phase p: rows kp + 8j + b, word tn.
  uint2 br[KB];
  auto fetch = [&](int p) {
    const int64_t kp = (int64_t)p * P32;
    const int rows = (int)imin64(d.k - kp, P32);
    const __amdgpu_buffer_rsrc_t rb = make_rsrc(d.B + kp * d.ldb + tn, (int64_t)(rows - 1) * ldb_b + 8);
#pragma unroll
    for (int b = 0; b < KB; ++b) br[b] = bload2(rb, (int)(8 * lr + b) * ldb_b);
  };
  auto build = [&](int buf) {
    const uint32_t hb = 2u * (uint32_t)w + ((uint32_t)L >> 5);     // index bits 3..7
    uint2 v = make_uint2(0, 0);
#pragma unroll
    for (int b = 3; b < KB; ++b)
      if ((hb >> (b - 3)) & 1u) v = make_uint2(v.x ^ br[b].x, v.y ^ br[b].y);
    char* dst = tab + ((uint32_t)buf << 16) + lr * 8;
    *reinterpret_cast<uint2*>(dst + (hb << 3) * 256) = v;
#pragma unroll
    for (int i = 1; i < 8; ++i) {
      const int c = __builtin_ctz(i);
      v = make_uint2(v.x ^ br[c].x, v.y ^ br[c].y);
      *reinterpret_cast<uint2*>(dst + ((hb << 3) | (uint32_t)(i ^ (i >> 1))) * 256) = v;
    }
  };
  if (nphases > 0) {
    load_a(0, ax);
    fetch(0);
    build(0);
  }
  __syncthreads();

  // Lookup address, low byte: (8q + (s ^ rx)) * 8 = base ^ (s * 8), base = (8q + rx) * 8.
  const uint32_t lb0 = (((uint32_t)q << 3) | rx) << 3;
  auto phase = [&](int p, uint2 (&cur)[RPT], uint2 (&nxt)[RPT]) {
    if (p + 1 < nphases) {
      fetch(p + 1);
      load_a(p + 1, nxt);
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const uint32_t lo = __builtin_amdgcn_perm(cur[i].y, cur[i].x, sel_lo);
      const uint32_t hi = __builtin_amdgcn_perm(cur[i].y, cur[i].x, sel_hi);
      cur[i] = make_uint2(lo, hi);
    }
    const uint32_t lbase = lb0 | ((uint32_t)(p & 1) << 16);
#pragma unroll
    for (int st = 0; st < 8; ++st) {
      const uint32_t lb = lbase ^ ((uint32_t)st << 3);
      constexpr uint32_t base_sel = 0x0c020400u;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const uint32_t src = st < 4 ? cur[i].x : cur[i].y;
        const uint32_t a = __builtin_amdgcn_perm(src, lb, base_sel + ((uint32_t)(st & 3) << 8));
        const uint2 t = *reinterpret_cast<const uint2*>(tab + a);
        acc[i] = make_uint2(acc[i].x ^ t.x, acc[i].y ^ t.y);
      }
      // Register fence every two steps: at most 2*RPT lookups in flight.
      if (st & 1) {
#pragma unroll
        for (int i = 0; i < RPT; ++i) asm volatile("" : "+v"(acc[i].x), "+v"(acc[i].y));
      }
    }
    if (p + 1 < nphases) build((p & 1) ^ 1);
    __syncthreads();
  };
  for (int p = 0; p < nphases; p += 2) {
    phase(p, ax, ay);
    if (p + 1 < nphases) phase(p + 1, ay, ax);
  }

  // Combine the four quarters of each row (lanes 4r..4r+3) and let quarter 0 store.
  const uint64_t tail = ((d.n & 63) && tn == words(d.n) - 1) ? ((1ull << (d.n & 63)) - 1) : ~0ull;
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    uint32_t x = acc[i].x, y = acc[i].y;
    x ^= (uint32_t)__shfl_xor((int)x, 1);
    y ^= (uint32_t)__shfl_xor((int)y, 1);
    x ^= (uint32_t)__shfl_xor((int)x, 2);
    y ^= (uint32_t)__shfl_xor((int)y, 2);
    const int r = 16 * i + r16;
    if (q == 0 && (!EDGE || r < rows_here))
      store_word(d.C + (row0 + r) * d.ldc + tn, ((uint64_t)x | ((uint64_t)y << 32)) & tail, d.out);
  }
}

template <int WAVES, int RPT>
__device__ __forceinline__ void m4rm32_tile_any(const MulDesc& d, int tm, int tn, char* tab) {
  using T = Tile32<WAVES, RPT>;
  if ((int64_t)(tm + 1) * T::BM > d.m) m4rm32_tile<WAVES, RPT, true>(d, tm, tn, tab);
  else m4rm32_tile<WAVES, RPT, false>(d, tm, tn, tab);
}

// Tile policies: a tile family (tables per phase and tile width), its height and its table
// width KAPPA (index bits per table, Section 3.1).
template <int WAVES, int RW>
struct PolicyT1 {
  static constexpr int BM = WAVES * RW, TW = TILE_WORDS, NT = WAVES * 64, PR = KB;
  static constexpr int LDS_BYTES = 2 * TABLE_BYTES;
  __device__ __forceinline__ static void run(const MulDesc& d, int tm, int tn, char* tab) { m4rm_tile_any<WAVES, RW>(d, tm, tn, tab); }
};
template <int WAVES, int S, int INFL, int KAPPA = KB>
struct PolicyT2 {
  static constexpr int BM = Tile2<WAVES, S, KAPPA>::BM, TW = T2_WORDS, NT = WAVES * 64, PR = 2 * KAPPA;
  static constexpr int LDS_BYTES = 2 * TABLE_BYTES;
  __device__ __forceinline__ static void run(const MulDesc& d, int tm, int tn, char* tab) {
    m4rm2_tile_any<WAVES, S, INFL, KAPPA>(d, tm, tn, tab);
  }
};
template <int WAVES, int RPT>
struct PolicyT32 {
  static constexpr int BM = Tile32<WAVES, RPT>::BM, TW = 1, NT = WAVES * 64, PR = P32;
  static constexpr int LDS_BYTES = 2 * TABLE_BYTES;
  __device__ __forceinline__ static void run(const MulDesc& d, int tm, int tn, char* tab) { m4rm32_tile_any<WAVES, RPT>(d, tm, tn, tab); }
};
template <int WAVES, int S, int KAPPA = KB>
struct PolicyT4 {
  static constexpr int BM = Tile4<WAVES, S, KAPPA>::BM, TW = T4_WORDS, NT = WAVES * 64, PR = 4 * KAPPA;
  static constexpr int LDS_BYTES = 2 * TABLE_BYTES;
  __device__ __forceinline__ static void run(const MulDesc& d, int tm, int tn, char* tab) { m4rm4_tile_any<WAVES, S, KAPPA>(d, tm, tn, tab); }
};
template <int WAVES, int S, int KAPPA = KB>
struct PolicyT8 {
  static constexpr int BM = Tile8<WAVES, S, KAPPA>::BM, TW = T8_WORDS, NT = WAVES * 64, PR = 8 * KAPPA;
  static constexpr int LDS_BYTES = 2 * TABLE_BYTES;
  __device__ __forceinline__ static void run(const MulDesc& d, int tm, int tn, char* tab) { m4rm8_tile_any<WAVES, S, KAPPA>(d, tm, tn, tab); }
};

// Algorithm 1 as it stands, without the row blocking of Algorithm 2 (the ablation's first arm):
// for each 8-row stripe of B, one table of the 256 combinations of the stripe's rows serves every
// row of A, and C is read and written in global memory once per stripe (2mnk/64 bytes in all,
// which the blocked algorithms avoid).  Parallelised over blocks of C: a workgroup owns a
// BM-row x TW-word block, builds its own copy of the stripe's table restricted to its TW words
// (32 groups of 8 entries, each group a Gray walk in which every entry after the first costs one
// row addition), then adds T[x_j] into C[j] in global memory for every row j of its block.
// Lane w = tid % TW owns word w of the block, so each row's TW words are one coalesced segment.
struct PolicyAlg1 {
  static constexpr int BM = 512, TW = 8, NT = 256, PR = KB, LDS_BYTES = 256 * TW * 8;
  static constexpr int LANES = NT / TW, UNROLL = 4;
  __device__ __forceinline__ static void run(const MulDesc& d, int tm, int tn, char* tabc) {
    uint64_t* tab = reinterpret_cast<uint64_t*>(tabc);  // tab[x * TW + w]
    const int tid = threadIdx.x, w = tid % TW, lane = tid / TW;
    const int64_t Wn = words(d.n), col = (int64_t)tn * TW + w;
    const bool valid = col < Wn;
    const uint64_t tail = ((d.n & 63) && col == Wn - 1) ? ((1ull << (d.n & 63)) - 1) : ~0ull;
    const int64_t r0 = (int64_t)tm * BM;
    const int rows = (int)(d.m - r0 < BM ? d.m - r0 : BM);
    gword* cb = (gword*)(d.C + r0 * d.ldc + col);
    const uint8_t* ab = reinterpret_cast<const uint8_t*>(d.A + r0 * d.lda);
    if (d.out == OUT_STORE && valid)
      for (int r = lane; r < rows; r += LANES) cb[r * d.ldc] = 0;
    const int nstripes = (d.k + KB - 1) / KB;
    for (int p = 0; p < nstripes; ++p) {
      const int64_t kp = (int64_t)p * KB;
      {
        uint64_t brow[KB];
#pragma unroll
        for (int b = 0; b < KB; ++b) brow[b] = (valid && kp + b < d.k) ? d.B[(kp + b) * d.ldb + col] & tail : 0;
        uint64_t v = 0;
#pragma unroll
        for (int b = 3; b < KB; ++b)
          if ((lane >> (b - 3)) & 1) v ^= brow[b];
        tab[(lane << 3) * TW + w] = v;
#pragma unroll
        for (int i = 1; i < 8; ++i) {
          v ^= brow[__builtin_ctz(i)];
          tab[((lane << 3) | (i ^ (i >> 1))) * TW + w] = v;
        }
      }
      __syncthreads();
      if (valid) {
        // UNROLL rows per pass, all loads before the stores, so that the rows' loads overlap.
        for (int r = lane; r < rows; r += UNROLL * LANES) {
          uint32_t x[UNROLL];
          uint64_t c[UNROLL];
#pragma unroll
          for (int u = 0; u < UNROLL; ++u) {
            const int rr = r + u * LANES;
            x[u] = rr < rows ? ab[(int64_t)rr * d.lda * 8 + p] : 0;
            c[u] = (rr < rows && d.out != OUT_ATOMIC) ? cb[rr * d.ldc] : 0;
          }
#pragma unroll
          for (int u = 0; u < UNROLL; ++u) {
            const int rr = r + u * LANES;
            if (rr < rows) {
              const uint64_t t = tab[x[u] * TW + w];
              if (d.out == OUT_ATOMIC) {
                if (t)
                  atomicXor(reinterpret_cast<unsigned long long*>(d.C + (r0 + rr) * d.ldc + col),
                            (unsigned long long)t);
              } else {
                cb[rr * d.ldc] = c[u] ^ t;
              }
            }
          }
        }
      }
      __syncthreads();
    }
  }
};

// Up to kMaxGroup products in one launch, descriptors passed by value (no device
// staging, so the launch can be captured into a graph as is).  Workgroup b belongs to
// the product i with tile_start[i] <= b < tile_start[i+1].
template <class P>
__global__ __launch_bounds__(P::NT) void m4rm_group(GroupArgs g) {
  __shared__ uint4 tab[P::LDS_BYTES / 16];
  const int b = blockIdx.x;
  const int t = b < g.remap_n ? xcd_remap(b, g.remap_n) : b;
  int i = 0;
  while (i + 1 < g.count && g.tile_start[i + 1] <= t) ++i;
  const MulDesc& d = g.d[i];
  const int local = t - g.tile_start[i];
  const int tiles_n = (int)((words(d.n) + P::TW - 1) / P::TW);
  P::run(d, local / tiles_n, local % tiles_n, reinterpret_cast<char*>(tab));
}

// Table widths: 8 for every tile; the tiles of at most 1024 rows (the ones short enough for
// the table build to matter, and the persistent kernel's) also 4 to 7.
constexpr int kKappaMin = 4;
constexpr int kNumKappa = KB - kKappaMin + 1;

struct Variant {
  int threads, bm, tw, pr;                // workgroup size, tile rows, tile width in words, B rows per phase at 8
  void (*group[kNumKappa])(GroupArgs);    // by table width - kKappaMin; null where the tile lacks it
};

template <class P>
Variant variant8() {
  return {P::NT, P::BM, P::TW, P::PR, {nullptr, nullptr, nullptr, nullptr, m4rm_group<P>}};
}
template <template <int> class F>
Variant variantk() {
  return {F<KB>::NT, F<KB>::BM, F<KB>::TW, F<KB>::PR,
          {m4rm_group<F<4>>, m4rm_group<F<5>>, m4rm_group<F<6>>, m4rm_group<F<7>>, m4rm_group<F<8>>}};
}

using V0 = PolicyT2<16, 12, 2>;   // t=2, BM 1536 x 1024 columns
template <int K> using V1 = PolicyT2<16, 8, 2, K>;   // t=2, BM 1024
template <int K> using V2 = PolicyT2<16, 4, 4, K>;   // t=2, BM 512
template <int K> using V3 = PolicyT2<16, 2, 2, K>;   // t=2, BM 256
template <int K> using V4 = PolicyT2<16, 1, 1, K>;   // t=2, BM 128
using V5 = PolicyT1<16, 48>;      // t=1, BM 768 x 2048 columns
using V6 = PolicyT1<16, 32>;      // t=1, BM 512
using V7 = PolicyT2<8, 4, 4>;     // t=2, BM 256, 8 waves
using V8 = PolicyT1<8, 32>;       // t=1, BM 256, 8 waves
using V9 = PolicyT1<4, 32>;       // t=1, BM 128, 4 waves
using V10 = PolicyT2<16, 11, 2>;  // t=2, BM 1408: six tiles cover 8192 rows
using V11 = PolicyT8<16, 4>;      // t=8, BM 2048 x 256 columns (narrow products)
template <int K> using V12 = PolicyT8<16, 2, K>;     // t=8, BM 1024
template <int K> using V13 = PolicyT8<16, 1, K>;     // t=8, BM 512
using V14 = PolicyT32<16, 4>;     // t=32, BM 1024 x 64 columns (matrix-vector, n <= 64)
using V15 = PolicyT32<16, 2>;     // t=32, BM 512
using V16 = PolicyT4<16, 8>;      // t=4, BM 2048 x 512 columns: four tiles cover 8192 rows
using V17 = PolicyT4<16, 6>;      // t=4, BM 1536
template <int K> using V18 = PolicyT4<16, 4, K>;     // t=4, BM 1024
template <int K> using V19 = PolicyT4<16, 2, K>;     // t=4, BM 512
template <int K> using V20 = PolicyT4<16, 1, K>;     // t=4, BM 256
using V21 = PolicyAlg1;           // Algorithm 1: one table per stripe for all m rows, C in global memory
using V22 = PolicyT8<16, 8>;      // t=8, BM 4096 x 256 columns: two tiles cover 8192 rows
const Variant kVariants[] = {variant8<V0>(), variantk<V1>(), variantk<V2>(), variantk<V3>(), variantk<V4>(),
                             variant8<V5>(), variant8<V6>(), variant8<V7>(), variant8<V8>(), variant8<V9>(),
                             variant8<V10>(), variant8<V11>(), variantk<V12>(), variantk<V13>(), variant8<V14>(),
                             variant8<V15>(), variant8<V16>(), variant8<V17>(), variantk<V18>(), variantk<V19>(),
                             variantk<V20>(), variant8<V21>(), variant8<V22>()};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

// The persistent kernel's tables, at file scope so that the tile functions below address
// them as LDS directly.
__shared__ uint4 g_ptab[2 * TABLE_BYTES / 16];

__device__ __forceinline__ int64_t uniform64(int64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) { return reinterpret_cast<T*>(uniform64((int64_t)p)); }

// One tile of the persistent kernel, compiled as a function of its own: inlined together, the
// tile families' register allocations merge and spill, while each alone fits.  Arguments of a
// device function arrive in vector registers; the descriptor is uniform, so its fields are
// moved back to scalar registers before use.
template <class P>
__device__ __noinline__ void persistent_tile(MulDesc d, int tm, int tn) {
  MulDesc u;
  u.A = uniform_ptr(d.A);
  u.B = uniform_ptr(d.B);
  u.C = uniform_ptr(d.C);
  u.lda = uniform64(d.lda);
  u.ldb = uniform64(d.ldb);
  u.ldc = uniform64(d.ldc);
  u.m = __builtin_amdgcn_readfirstlane(d.m);
  u.k = __builtin_amdgcn_readfirstlane(d.k);
  u.n = __builtin_amdgcn_readfirstlane(d.n);
  u.out = __builtin_amdgcn_readfirstlane(d.out);
  P::run(u, __builtin_amdgcn_readfirstlane(tm), __builtin_amdgcn_readfirstlane(tn), reinterpret_cast<char*>(g_ptab));
}

template <template <int> class F>
__device__ __forceinline__ void run_kappa(int kappa, const MulDesc& d, int tm, int tn) {
  switch (kappa) {
    case 4: persistent_tile<F<4>>(d, tm, tn); break;
    case 5: persistent_tile<F<5>>(d, tm, tn); break;
    case 6: persistent_tile<F<6>>(d, tm, tn); break;
    case 7: persistent_tile<F<7>>(d, tm, tn); break;
    default: persistent_tile<F<8>>(d, tm, tn); break;
  }
}

// Persistent batch kernel: one workgroup per compute unit pulls tile items from an
// atomic queue (ordered longest first) until it runs dry; every item names its product,
// one of the 16-wave variants (two tables per phase up to 1024 rows, four or eight up to
// 2048) and its table width (variant | width << 8; the tiles of more than 1024 rows only
// take 8).  Each tile ends on a barrier, so LDS is free for the next item.
__global__ __launch_bounds__(1024) void m4rm_persistent(const MulDesc* __restrict__ ds,
                                                        const BatchItem* __restrict__ items, int nitems,
                                                        int* __restrict__ counter) {
  __shared__ int next;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(counter, 1);
    __syncthreads();
    const int i = next;
    __syncthreads();
    if (i >= nitems) break;
    const BatchItem it = items[i];
    const MulDesc d = ds[it.desc];
    const int kappa = it.variant >> 8;
    switch (it.variant & 0xff) {
      case 1: run_kappa<V1>(kappa, d, it.tm, it.tn); break;
      case 2: run_kappa<V2>(kappa, d, it.tm, it.tn); break;
      case 3: run_kappa<V3>(kappa, d, it.tm, it.tn); break;
      case 12: run_kappa<V12>(kappa, d, it.tm, it.tn); break;
      case 13: run_kappa<V13>(kappa, d, it.tm, it.tn); break;
      case 18: run_kappa<V18>(kappa, d, it.tm, it.tn); break;
      case 19: run_kappa<V19>(kappa, d, it.tm, it.tn); break;
      case 20: run_kappa<V20>(kappa, d, it.tm, it.tn); break;
      case 16: persistent_tile<V16>(d, it.tm, it.tn); break;
      case 17: persistent_tile<V17>(d, it.tm, it.tn); break;
      case 11: persistent_tile<V11>(d, it.tm, it.tn); break;
      default: run_kappa<V4>(kappa, d, it.tm, it.tn); break;
    }
  }
}

__global__ void reset_counter(int* c) { *c = 0; }

// Index expansion of A for a table narrower than 8 bits (Section 3: with a table of kappa
// index bits, row r's stripe j is selected by bits kappa*j .. kappa*j + kappa - 1 of A's row).
// Byte j of row r of X holds that field (its bit 0 = column kappa*j); bits of A at or past k
// read as zero and X's bytes past ceil(k / kappa), up to the row's ldx words, are written 0, so
// the M4RM tiles read one index byte per lookup whatever the width.  One dword of X per thread,
// the op's dwords spread over all of the launch's threads (products of a batch are small, and
// a block per row would leave most threads idle).
__device__ __forceinline__ void expand_rows(const ExpandOp& o) {
  const int dws = (int)(2 * o.ldx);
  const int kw = (int)words(o.k);
  const int64_t total = (int64_t)o.m * dws;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e < 0xffffffffll ? (int64_t)((uint32_t)e / (uint32_t)dws) : e / dws;
    const int j = (int)(e - r * dws);
    const uint64_t* row = o.A + r * o.lda;
    uint32_t* dst = reinterpret_cast<uint32_t*>(o.X + r * o.ldx);
    {
      uint32_t out = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t bit = (int64_t)(4 * j + q) * o.kappa;
        if (bit < o.k) {
          const int w = (int)(bit >> 6), sh = (int)(bit & 63);
          uint64_t v = row[w] >> sh;
          if (sh + o.kappa > 64 && w + 1 < kw) v |= row[w + 1] << (64 - sh);
          const int64_t nb = imin64(o.kappa, o.k - bit);
          out |= (uint32_t)(v & ((1ull << nb) - 1)) << (8 * q);
        }
      }
      dst[j] = out;
    }
  }
}

constexpr int kExpandOps = 64;
struct ExpandArgs {
  ExpandOp op[kExpandOps];
  int count;
};

__global__ __launch_bounds__(256) void expand_group(ExpandArgs a) { expand_rows(a.op[blockIdx.y]); }
__global__ __launch_bounds__(256) void expand_list(const ExpandOp* __restrict__ ops) { expand_rows(ops[blockIdx.y]); }

const Variant& variant_of(int v) { return kVariants[(v < 0 || v >= kNumVariants) ? 0 : v]; }

// Blocks per op: enough for the largest op's dwords (256 per block), at most 1024.
unsigned expand_grid_x(int64_t max_dwords) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((max_dwords + 255) / 256, 1024));
}

}  // namespace

int m4rm_num_variants() { return kNumVariants; }
int m4rm_tile_rows(int variant) { return variant_of(variant).bm; }
int m4rm_tile_words(int variant) { return variant_of(variant).tw; }
int m4rm_phase_rows(int variant, int kappa) { return variant_of(variant).pr / KB * kappa; }
bool m4rm_has_kappa(int variant, int kappa) {
  return kappa >= kKappaMin && kappa <= KB && variant >= 0 && variant < kNumVariants &&
         variant_of(variant).group[kappa - kKappaMin] != nullptr;
}

int64_t m4rm_tiles(const MulDesc& d, int variant) {
  const int64_t bm = variant_of(variant).bm, tw = variant_of(variant).tw;
  return ((d.m + bm - 1) / bm) * ((words(d.n) + tw - 1) / tw);
}

int64_t m4rm_expanded_ld(int64_t k, int kappa) { return ((k + kappa - 1) / kappa + 7) / 8; }

gf2_status m4rm_expand(const ExpandOp* ops, int n, hipStream_t s) {
  for (int i = 0; i < n; i += kExpandOps) {
    ExpandArgs a;
    a.count = std::min(kExpandOps, n - i);
    int64_t dwords = 0;
    for (int j = 0; j < a.count; ++j) {
      a.op[j] = ops[i + j];
      dwords = std::max<int64_t>(dwords, (int64_t)a.op[j].m * 2 * a.op[j].ldx);
    }
    hipLaunchKernelGGL(expand_group, dim3(expand_grid_x(dwords), (unsigned)a.count), dim3(256), 0, s, a);
    gf2_status st = hip_check(hipGetLastError(), "expand_group launch");
    if (st != GF2_OK) return st;
  }
  return GF2_OK;
}

gf2_status m4rm_expand_list(const ExpandOp* dev_ops, int n, int64_t max_dwords, hipStream_t s) {
  for (int i = 0; i < n; i += 65535) {   // grid y limit
    const int c = std::min(65535, n - i);
    hipLaunchKernelGGL(expand_list, dim3(expand_grid_x(max_dwords), (unsigned)c), dim3(256), 0, s, dev_ops + i);
    gf2_status st = hip_check(hipGetLastError(), "expand_list launch");
    if (st != GF2_OK) return st;
  }
  return GF2_OK;
}

gf2_status m4rm_launch_group(const MulDesc* descs, int count, int variant, hipStream_t s, int tail, int kappa) {
  if (!m4rm_has_kappa(variant, kappa))
    return set_error(GF2_ERR_UNSUPPORTED, "M4RM variant %d has no %d-bit tables", variant, kappa);
  // A narrower table reads A's index expansion, whose rows the tiles address with 32-bit offsets.
  if (kappa < KB)
    for (int i = 0; i < count; ++i)
      if (descs[i].lda >= (int64_t(1) << 20))
        return set_error(GF2_ERR_UNSUPPORTED, "%d-bit tables need k below %lld", kappa, (long long)kappa << 23);
  // The one-word tile addresses 256 rows of B per phase with 32-bit offsets: for B rows of
  // 2^20 words or more the eight-table 512-row tile (same bits) runs instead.
  if (variant_of(variant).pr == P32)
    for (int i = 0; i < count; ++i)
      if (descs[i].ldb >= (int64_t(1) << 20)) {
        variant = 13;
        break;
      }
  // The four-table tiles address up to 128 rows of A per wave the same way: for A rows of
  // 2^20 words or more the 1408-row two-table tile runs instead; the 4096-row eight-table
  // tile (256 rows per wave) hands such an A to the 2048-row one.
  if (variant_of(variant).tw == T4_WORDS)
    for (int i = 0; i < count; ++i)
      if (descs[i].lda >= (int64_t(1) << 20)) {
        variant = 10;
        break;
      }
  if (variant == 22)
    for (int i = 0; i < count; ++i)
      if (descs[i].lda >= (int64_t(1) << 20)) {
        variant = 11;
        break;
      }
  const Variant& v = variant_of(variant);
  const int tail_begin = count - (tail > 0 ? tail : 0);
  int i = 0;
  while (i < count) {
    GroupArgs g;
    g.count = 0;
    g.remap_n = -1;
    int64_t total = 0;
    for (; i < count && g.count < kMaxGroup; ++i) {
      const int64_t t = m4rm_tiles(descs[i], variant);
      if (t == 0) continue;
      if (i >= tail_begin && g.remap_n < 0) g.remap_n = (int)total;
      g.d[g.count] = descs[i];
      g.tile_start[g.count] = (int)total;
      ++g.count;
      total += t;
      if (total > INT32_MAX) return set_error(GF2_ERR_UNSUPPORTED, "m4rm: too many tiles in one launch");
    }
    if (g.count == 0) continue;
    g.tile_start[g.count] = (int)total;
    if (g.remap_n < 0) g.remap_n = (int)total;
    double work = 0;
    for (int j = 0; j < g.count; ++j)
      work += (double)g.d[j].m * ((g.d[j].k + kappa - 1) / kappa) * (double)words(g.d[j].n);
    TraceScope trace(GF2_TRACE_M4RM, g.count, work, s);
    hipLaunchKernelGGL(v.group[kappa - kKappaMin], dim3((unsigned)total), dim3(v.threads), 0, s, g);
    gf2_status st = hip_check(hipGetLastError(), "m4rm_group launch");
    if (st != GF2_OK) return st;
  }
  return GF2_OK;
}

bool m4rm_batchable(int variant) {
  switch (variant) {
    case 1: case 2: case 3: case 4: case 11: case 12: case 13: case 16: case 17: case 18: case 19: case 20: return true;
    default: return false;
  }
}

gf2_status m4rm_launch_persistent(const MulDesc* dev_descs, const BatchItem* dev_items, int nitems, int* dev_counter,
                                  int grid, hipStream_t s) {
  hipLaunchKernelGGL(reset_counter, dim3(1), dim3(1), 0, s, dev_counter);
  gf2_status st = hip_check(hipGetLastError(), "reset_counter launch");
  if (st != GF2_OK || nitems == 0) return st;
  hipLaunchKernelGGL(m4rm_persistent, dim3(grid), dim3(1024), 0, s, dev_descs, dev_items, nitems, dev_counter);
  return hip_check(hipGetLastError(), "m4rm_persistent launch");
}

}  // namespace gf2
