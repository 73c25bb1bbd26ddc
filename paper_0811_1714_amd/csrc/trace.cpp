// Launch tracing: event pairs around kernel launches, read back on demand.
#include <atomic>
#include <mutex>
#include <vector>

#include "gf2_internal.h"

namespace gf2 {
namespace {
struct Rec {
  int kind, items;
  double work;
  hipEvent_t e0, e1;
};
std::atomic<bool> g_on{false};
thread_local bool g_suspended = false;
std::mutex g_mu;
std::vector<Rec> g_recs;
}  // namespace

bool trace_on() { return g_on.load(std::memory_order_relaxed) && !g_suspended; }
void trace_suspend(bool on) { g_suspended = on; }

TraceScope::TraceScope(int kind, int items, double work, hipStream_t s) : kind_(kind), items_(items), work_(work), s_(s) {
  if (!trace_on()) return;
  if (hipEventCreate(&e0_) != hipSuccess) { e0_ = nullptr; return; }
  if (hipEventRecord(e0_, s_) != hipSuccess) { (void)hipEventDestroy(e0_); e0_ = nullptr; }
}

TraceScope::~TraceScope() {
  if (!e0_) return;
  hipEvent_t e1 = nullptr;
  if (hipEventCreate(&e1) != hipSuccess || hipEventRecord(e1, s_) != hipSuccess) {
    (void)hipEventDestroy(e0_);
    if (e1) (void)hipEventDestroy(e1);
    return;
  }
  std::lock_guard<std::mutex> g(g_mu);
  g_recs.push_back(Rec{kind_, items_, work_, e0_, e1});
}

}  // namespace gf2

using namespace gf2;

extern "C" {

gf2_status gf2_trace_enable(int32_t on) {
  g_on.store(on != 0);
  return GF2_OK;
}

gf2_status gf2_trace_read(gf2_trace_record* out, int64_t max, int64_t* count) {
  if (!count || (max > 0 && !out)) return set_error(GF2_ERR_INVALID_ARG, "gf2_trace_read: null output");
  std::lock_guard<std::mutex> g(g_mu);
  int64_t n = 0;
  for (const Rec& r : g_recs) {
    if (n >= max) break;
    gf2_status st = hip_check(hipEventSynchronize(r.e1), "hipEventSynchronize");
    if (st != GF2_OK) return st;
    float ms = 0;
    st = hip_check(hipEventElapsedTime(&ms, r.e0, r.e1), "hipEventElapsedTime");
    if (st != GF2_OK) return st;
    out[n++] = gf2_trace_record{r.kind, r.items, r.work, (double)ms};
  }
  *count = n;
  return GF2_OK;
}

void gf2_trace_clear(void) {
  std::lock_guard<std::mutex> g(g_mu);
  for (const Rec& r : g_recs) {
    (void)hipEventDestroy(r.e0);
    (void)hipEventDestroy(r.e1);
  }
  g_recs.clear();
}

}  // extern "C"
