// Candidate schedules and the schedule policy used by single and batched products.
#include "gf2_internal.h"

namespace gf2 {
namespace {

// The candidate list: M4RM tile heights (the persistent-kernel variants first), split-K
// for tall-narrow work, one Strassen-Winograd level, the 1536-row tile, and the two
// other base cases.  Index order is part of the ABI (schedule model outputs follow it).
const gf2_schedule kCandidates[] = {
    {GF2_KERNEL_M4RM, 1, 0, 1},      // 0: t=2, 1024 rows
    {GF2_KERNEL_M4RM, 2, 0, 1},      // 1: t=2, 512 rows
    {GF2_KERNEL_M4RM, 3, 0, 1},      // 2: t=2, 256 rows
    {GF2_KERNEL_M4RM, 4, 0, 1},      // 3: t=2, 128 rows
    {GF2_KERNEL_M4RM, 2, 0, 4},      // 4: 512 rows, k in 4 slices
    {GF2_KERNEL_M4RM, 3, 0, 16},     // 5: 256 rows, k in 16 slices
    {GF2_KERNEL_M4RM, 1, 1024, 1},   // 6: Strassen-Winograd above 1024, 1024-row leaves
    {GF2_KERNEL_M4RM, 0, 0, 1},      // 7: t=2, 1536 rows
    {GF2_KERNEL_MFMA, 0, 0, 1},      // 8: int8 matrix core
    {GF2_KERNEL_CUBIC, 0, 0, 1},     // 9: popcount
};
constexpr int kNumCandidates = sizeof(kCandidates) / sizeof(kCandidates[0]);

}  // namespace

int num_candidates() { return kNumCandidates; }
const gf2_schedule& candidate(int i) { return kCandidates[i]; }

// The fixed heuristic (no tuning data): among the persistent-kernel M4RM tiles, the one
// that minimises (tiles) x (16-row phases) x (rows per tile + the table build, counted
// as 256 row lookups per phase) -- the paper's trade-off between block size and the
// cost of regenerating the tables (Section 3.2), with LDS in place of cache.
int choose_candidate(int64_t m, int64_t k, int64_t n) {
  int best = 0;
  double best_cost = 0;
  for (int c = 0; c <= 3; ++c) {
    const gf2_schedule& s = kCandidates[c];
    const int64_t bm = m4rm_tile_rows(s.variant), tw = m4rm_tile_words(s.variant);
    const double tiles = (double)((m + bm - 1) / bm) * (double)((words(n) + tw - 1) / tw);
    const double cost = tiles * (double)((k + 15) / 16) * (double)(bm + 256);
    if (c == 0 || cost < best_cost) { best = c; best_cost = cost; }
  }
  return best;
}

}  // namespace gf2

using namespace gf2;

extern "C" {

int32_t gf2_num_candidates(void) { return kNumCandidates; }

gf2_status gf2_candidate(int32_t index, gf2_schedule* out) {
  if (!out || index < 0 || index >= kNumCandidates)
    return set_error(GF2_ERR_INVALID_ARG, "candidate index %d out of range [0, %d)", index, kNumCandidates);
  *out = kCandidates[index];
  return GF2_OK;
}

}  // extern "C"
