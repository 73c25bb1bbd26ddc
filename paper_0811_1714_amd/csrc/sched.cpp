// Candidate schedules and the schedule policy used by single and batched products.
#include <cmath>
#include <mutex>
#include <vector>

#include "gf2_internal.h"

namespace gf2 {
namespace {

// The candidate list: every tile the persistent batch kernel runs (two-table tiles of 1024 to
// 128 rows, four-table tiles of 2048 to 256, eight-table tiles of 2048 to 512) with 8-bit
// tables, the short ones also with 7- to 5-bit tables (a product of few rows builds its tables
// for few lookups), k-split and one-level Strassen-Winograd forms, and schedules that only run
// as grouped launches (the 1536-row two-table tile, the int8 matrix core, the popcount kernel).
// Index order is part of the ABI (schedule model outputs follow it); later additions are appended.
const gf2_schedule kCandidates[] = {
    {GF2_KERNEL_M4RM, 1, 0, 1, 0, 8},      //  0: t=2, 1024 rows x 1024 columns
    {GF2_KERNEL_M4RM, 2, 0, 1, 0, 8},      //  1: t=2, 512 rows
    {GF2_KERNEL_M4RM, 3, 0, 1, 0, 8},      //  2: t=2, 256 rows
    {GF2_KERNEL_M4RM, 4, 0, 1, 0, 8},      //  3: t=2, 128 rows
    {GF2_KERNEL_M4RM, 18, 0, 1, 0, 8},     //  4: t=4, 1024 rows x 512 columns
    {GF2_KERNEL_M4RM, 19, 0, 1, 0, 8},     //  5: t=4, 512 rows
    {GF2_KERNEL_M4RM, 20, 0, 1, 0, 8},     //  6: t=4, 256 rows
    {GF2_KERNEL_M4RM, 12, 0, 1, 0, 8},     //  7: t=8, 1024 rows x 256 columns
    {GF2_KERNEL_M4RM, 13, 0, 1, 0, 8},     //  8: t=8, 512 rows
    {GF2_KERNEL_M4RM, 4, 0, 1, 0, 7},      //  9: t=2, 128 rows, 7-bit tables
    {GF2_KERNEL_M4RM, 4, 0, 1, 0, 6},      // 10: t=2, 128 rows, 6-bit tables
    {GF2_KERNEL_M4RM, 4, 0, 1, 0, 5},      // 11: t=2, 128 rows, 5-bit tables
    {GF2_KERNEL_M4RM, 3, 0, 1, 0, 7},      // 12: t=2, 256 rows, 7-bit tables
    {GF2_KERNEL_M4RM, 3, 0, 1, 0, 6},      // 13: t=2, 256 rows, 6-bit tables
    {GF2_KERNEL_M4RM, 20, 0, 1, 0, 7},     // 14: t=4, 256 rows, 7-bit tables
    {GF2_KERNEL_M4RM, 20, 0, 1, 0, 6},     // 15: t=4, 256 rows, 6-bit tables
    {GF2_KERNEL_M4RM, 13, 0, 1, 0, 7},     // 16: t=8, 512 rows, 7-bit tables
    {GF2_KERNEL_M4RM, 13, 0, 1, 0, 6},     // 17: t=8, 512 rows, 6-bit tables
    {GF2_KERNEL_M4RM, 2, 0, 4, 0, 8},      // 18: t=2, 512 rows, k in 4 slices
    {GF2_KERNEL_M4RM, 3, 0, 16, 0, 8},     // 19: t=2, 256 rows, k in 16 slices
    {GF2_KERNEL_M4RM, 19, 0, 4, 0, 8},     // 20: t=4, 512 rows, k in 4 slices
    {GF2_KERNEL_M4RM, 1, 1024, 1, 0, 8},   // 21: Strassen-Winograd above 1024, t=2 1024-row leaves
    {GF2_KERNEL_M4RM, 18, 1024, 1, 0, 8},  // 22: Strassen-Winograd above 1024, t=4 1024-row leaves
    {GF2_KERNEL_M4RM, 0, 0, 1, 0, 8},      // 23: t=2, 1536 rows (grouped launch)
    {GF2_KERNEL_M4RM, 16, 0, 1, 0, 8},     // 24: t=4, 2048 rows
    {GF2_KERNEL_MFMA, 0, 0, 1, 0, 8},      // 25: int8 matrix core
    {GF2_KERNEL_CUBIC, 0, 0, 1, 0, 8},     // 26: popcount
    {GF2_KERNEL_M4RM, 17, 0, 1, 0, 8},     // 27: t=4, 1536 rows
    {GF2_KERNEL_M4RM, 11, 0, 1, 0, 8},     // 28: t=8, 2048 rows x 256 columns
};
constexpr int kNumCandidates = sizeof(kCandidates) / sizeof(kCandidates[0]);

}  // namespace

int num_candidates() { return kNumCandidates; }
const gf2_schedule& candidate(int i) { return kCandidates[i]; }

// The fixed heuristic (no tuning data): among the persistent-kernel tiles with 8-bit tables,
// the one that minimises (tiles) x (barrier phases) x (tile rows + the table build, counted as
// 256 rows) -- the paper's trade-off between block size and the cost of regenerating the
// tables (Section 3.2), with LDS in place of cache.  Every tile family reads 256 B of tables
// per row and phase and builds 64 KiB per phase; t tables per phase cover 8t rows of B and a
// tile 2048/t columns wide.
int fixed_candidate(int64_t m, int64_t k, int64_t n) {
  int best = 0;
  double best_cost = 0;
  for (int c : {0, 1, 2, 3, 4, 5, 6, 7, 8, 24, 27, 28}) {
    const gf2_schedule& s = kCandidates[c];
    const int64_t bm = m4rm_tile_rows(s.variant), tw = m4rm_tile_words(s.variant), pr = m4rm_phase_rows(s.variant);
    const double tiles = (double)((m + bm - 1) / bm) * (double)((words(n) + tw - 1) / tw);
    const double cost = tiles * (double)((k + pr - 1) / pr) * (double)(bm + 256);
    if (best_cost == 0 || cost < best_cost) { best = c; best_cost = cost; }
  }
  return best;
}

// ---- schedule model: host copy for single products, device copy for batches ----
namespace {
std::mutex g_model_mu;
std::vector<float> g_model;
float g_norm[8] = {0, 0, 0, 0, 1, 1, 1, 1};
float* g_model_dev = nullptr;
int g_model_dev_id = -1;
}  // namespace

bool model_available() {
  std::lock_guard<std::mutex> g(g_model_mu);
  return !g_model.empty();
}

void model_features(int64_t m, int64_t k, int64_t n, double density, float* x) {
  const double raw[4] = {std::log2((double)(m > 0 ? m : 1)), std::log2((double)(k > 0 ? k : 1)),
                         std::log2((double)(n > 0 ? n : 1)), density};
  for (int i = 0; i < 4; ++i) x[i] = (float)((raw[i] - g_norm[i]) / (g_norm[4 + i] != 0 ? g_norm[4 + i] : 1.0f));
}

bool model_predict(int64_t m, int64_t k, int64_t n, double density, float* out) {
  std::lock_guard<std::mutex> g(g_model_mu);
  if (g_model.empty()) return false;
  float x[4];
  model_features(m, k, n, density, x);
  mlp_forward_host(g_model.data(), x, 2 * kNumCandidates, out);
  return true;
}

int model_or_fixed(int pick, float y_pick, int fixed, float y_fixed) {
  // The model's outputs are predicted natural-log times: its pick must be predicted at least
  // kModelBatchMargin faster than the fixed rule's candidate to replace it.
  static const float kLogKeep = (float)std::log(1.0 - kModelBatchMargin);
  if (pick < 0 || pick == fixed) return fixed;
  return y_pick - y_fixed < kLogKeep ? pick : fixed;
}

// Device inference for many products: the batch head's argmin over the allowed candidates,
// kept only where it beats the fixed rule's candidate (fixed[b]) by the margin above.
gf2_status model_choose_batch(const std::vector<float>& feats_raw, const uint8_t* allowed_host,
                              const std::vector<int>& fixed, std::vector<int>& out) {
  const int64_t nb = (int64_t)feats_raw.size() / 4;
  out.assign(nb, -1);
  std::lock_guard<std::mutex> g(g_model_mu);
  if (g_model.empty() || nb == 0) return GF2_OK;
  int dev = 0;
  gf2_status r = hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (r != GF2_OK) return r;
  if (g_model_dev && g_model_dev_id != dev) {
    (void)hipFree(g_model_dev);
    g_model_dev = nullptr;
  }
  if (!g_model_dev) {
    if (hipMalloc(&g_model_dev, g_model.size() * sizeof(float)) != hipSuccess) {
      g_model_dev = nullptr;
      return set_error(GF2_ERR_ALLOC, "hipMalloc for the schedule model failed");
    }
    if ((r = hip_check(hipMemcpy(g_model_dev, g_model.data(), g_model.size() * sizeof(float),
                                 hipMemcpyHostToDevice), "hipMemcpy")) != GF2_OK)
      return r;
    g_model_dev_id = dev;
  }
  std::vector<float> x(nb * 4);
  for (int64_t b = 0; b < nb; ++b) {
    const double raw[4] = {feats_raw[4 * b], feats_raw[4 * b + 1], feats_raw[4 * b + 2], feats_raw[4 * b + 3]};
    for (int i = 0; i < 4; ++i)
      x[4 * b + i] = (float)((raw[i] - g_norm[i]) / (g_norm[4 + i] != 0 ? g_norm[4 + i] : 1.0f));
  }
  // One allocation: X, Y, acts, allowed (one byte per output, padded to 64), out.
  const int NO = 2 * kNumCandidates;   // batch outputs are the second half
  const size_t fX = nb * 4, fY = nb * NO, fA = 3 * nb * 64, mask_bytes = (NO + 63) & ~size_t(63);
  const size_t bytes = (fX + fY + fA) * sizeof(float) + mask_bytes + nb * sizeof(int32_t);
  char* buf = nullptr;
  if (hipMalloc(&buf, bytes) != hipSuccess) return set_error(GF2_ERR_ALLOC, "hipMalloc for model inference failed");
  float* dX = reinterpret_cast<float*>(buf);
  float* dY = dX + fX;
  float* dA = dY + fY;
  uint8_t* dAllowed = reinterpret_cast<uint8_t*>(dA + fA);
  int32_t* dOut = reinterpret_cast<int32_t*>(dAllowed + mask_bytes);
  std::vector<int32_t> host_out(nb);
  r = hip_check(hipMemcpy(dX, x.data(), fX * sizeof(float), hipMemcpyHostToDevice), "hipMemcpy");
  std::vector<uint8_t> mask(NO, 0);
  for (int c = 0; c < kNumCandidates; ++c) mask[kNumCandidates + c] = allowed_host[c];
  if (r == GF2_OK) r = hip_check(hipMemcpy(dAllowed, mask.data(), NO, hipMemcpyHostToDevice), "hipMemcpy");
  if (r == GF2_OK) r = mlp_forward(g_model_dev, dX, nb, NO, dY, dA, nullptr);
  if (r == GF2_OK) r = mlp_argmin(dY, nb, NO, dAllowed, dOut, nullptr);
  if (r == GF2_OK) r = hip_check(hipMemcpy(host_out.data(), dOut, nb * sizeof(int32_t), hipMemcpyDeviceToHost), "hipMemcpy");
  std::vector<float> y(r == GF2_OK ? fY : 0);
  if (r == GF2_OK) r = hip_check(hipMemcpy(y.data(), dY, fY * sizeof(float), hipMemcpyDeviceToHost), "hipMemcpy");
  (void)hipFree(buf);
  if (r != GF2_OK) return r;
  for (int64_t b = 0; b < nb; ++b) {
    const int p = host_out[b] >= kNumCandidates ? host_out[b] - kNumCandidates : -1;
    const float* yb = y.data() + b * NO + kNumCandidates;
    out[b] = p < 0 ? -1 : model_or_fixed(p, yb[p], fixed[b], yb[fixed[b]]);
  }
  return r;
}

bool batch_allowed(int c) {
  const gf2_schedule& s = kCandidates[c];
  return s.kernel == GF2_KERNEL_M4RM && m4rm_batchable(s.variant);
}

}  // namespace gf2

using namespace gf2;

extern "C" {

int32_t gf2_num_candidates(void) { return kNumCandidates; }

int64_t gf2_mlp_param_count(void) { return mlp_param_count(2 * kNumCandidates); }
int64_t gf2_mlp_scratch_floats(int64_t batch) { return batch < 0 ? 0 : mlp_scratch_floats(batch, 2 * kNumCandidates); }

gf2_status gf2_mlp_forward(const float* params, const float* X, int64_t batch, float* Y, float* acts, void* stream) {
  if (batch < 0 || (batch > 0 && (!params || !X || !Y || !acts)))
    return set_error(GF2_ERR_INVALID_ARG, "gf2_mlp_forward: bad arguments");
  return mlp_forward(params, X, batch, 2 * kNumCandidates, Y, acts, static_cast<hipStream_t>(stream));
}

gf2_status gf2_mlp_backward(const float* params, const float* X, int64_t batch, const float* acts, const float* Y,
                            const float* T, const float* M, float* grads, float* scratch, float* loss, void* stream) {
  if (batch < 0 || !params || !grads || !scratch || (batch > 0 && (!X || !acts || !Y || !T || !M)))
    return set_error(GF2_ERR_INVALID_ARG, "gf2_mlp_backward: bad arguments");
  return mlp_backward(params, X, batch, 2 * kNumCandidates, acts, Y, T, M, grads, scratch, loss,
                      static_cast<hipStream_t>(stream));
}

gf2_status gf2_mlp_adam(float* params, const float* grads, float* m, float* v, int64_t count, int32_t step, float lr,
                        float beta1, float beta2, float eps, void* stream) {
  if (count < 0 || step < 1 || (count > 0 && (!params || !grads || !m || !v)))
    return set_error(GF2_ERR_INVALID_ARG, "gf2_mlp_adam: bad arguments");
  return mlp_adam(params, grads, m, v, count, step, lr, beta1, beta2, eps, static_cast<hipStream_t>(stream));
}

gf2_status gf2_mlp_argmin(const float* Y, int64_t batch, const uint8_t* allowed, int32_t* out, void* stream) {
  if (batch < 0 || (batch > 0 && (!Y || !out))) return set_error(GF2_ERR_INVALID_ARG, "gf2_mlp_argmin: bad arguments");
  return mlp_argmin(Y, batch, 2 * kNumCandidates, allowed, out, static_cast<hipStream_t>(stream));
}

gf2_status gf2_set_model(const float* params, int64_t count, const float* norm) {
  bump_policy_epoch();
  std::lock_guard<std::mutex> g(g_model_mu);
  if (g_model_dev) {
    (void)hipFree(g_model_dev);
    g_model_dev = nullptr;
    g_model_dev_id = -1;
  }
  if (!params) {
    g_model.clear();
    return GF2_OK;
  }
  if (count != mlp_param_count(2 * kNumCandidates))
    return set_error(GF2_ERR_INVALID_ARG, "model has %lld parameters, expected %lld", (long long)count,
                     (long long)mlp_param_count(2 * kNumCandidates));
  g_model.assign(params, params + count);
  for (int i = 0; i < 8; ++i) g_norm[i] = norm ? norm[i] : (i < 4 ? 0.f : 1.f);
  return GF2_OK;
}

gf2_status gf2_candidate(int32_t index, gf2_schedule* out) {
  if (!out || index < 0 || index >= kNumCandidates)
    return set_error(GF2_ERR_INVALID_ARG, "candidate index %d out of range [0, %d)", index, kNumCandidates);
  *out = kCandidates[index];
  return GF2_OK;
}

}  // extern "C"
