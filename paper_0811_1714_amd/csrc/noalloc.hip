// gf2_mul_noalloc: a product whose workspace is a fixed device array of this library instead
// of memory it allocates, for callers that cannot allocate (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc).
//
// ``scratch`` below is a file-scope device array; every GPU the library runs on holds its own
// copy until the process ends.  In host code its name is only a stand-in for the symbol, so
// the device address is taken once per device with hipGetSymbolAddress (on the first call on
// that device, with it current) and that address is what the kernels receive.
#include <mutex>

#include "gf2_internal.h"

namespace gf2 {
namespace {

constexpr size_t kStaticScratchBytes = GF2_NOALLOC_SCRATCH_BYTES;
static_assert(kStaticScratchBytes % 256 == 0, "scratch size must keep 256-byte alignment");

__device__ __align__(256) uint64_t scratch[kStaticScratchBytes / 8];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint64_t* g_ptr[kMaxDevices] = {};

gf2_status scratch_address(uint64_t** out) {
  int dev = 0;
  gf2_status r = hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (r != GF2_OK) return r;
  if (dev < 0 || dev >= kMaxDevices) return set_error(GF2_ERR_UNSUPPORTED, "device id %d out of range", dev);
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_check(e, "hipGetSymbolAddress(scratch)");
    if (!p) return set_error(GF2_ERR_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_ptr[dev] = static_cast<uint64_t*>(p);
  }
  *out = g_ptr[dev];
  return GF2_OK;
}

}  // namespace
}  // namespace gf2

extern "C" gf2_status gf2_mul_noalloc(uint64_t* C, int64_t ldc, const uint64_t* A, int64_t lda, const uint64_t* B,
                                      int64_t ldb, int64_t m, int64_t k, int64_t n, int32_t accumulate,
                                      const gf2_schedule* sched, void* stream) {
  return gf2::mul_in_static(C, ldc, A, lda, B, ldb, m, k, n, accumulate != 0, sched, stream,
                            gf2::kStaticScratchBytes, gf2::scratch_address);
}
