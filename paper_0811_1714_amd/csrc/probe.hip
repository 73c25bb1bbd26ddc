// LDS bandwidth probes: the measured ceilings against which the M4RM kernels' table
// traffic is reported (their lookups read LDS, their table builds write it).
//
// Each workgroup of 1024 threads (16 waves, the M4RM tiles' shape) fills a 64 KiB LDS
// buffer, then issues unrolled accesses in the access pattern of the four-table tile:
// reads are ds_read_b128 where every 16 lanes cover all 64 banks (four 64 B table
// slices x four 16 B quarters of one 256 B entry), writes are ds_write_b32 of whole 256 B
// entries (64 lanes x 4 B), as the Gray-code build issues them.  The entry of each access is
// a compile-time constant folded into the instruction's offset, so one address register
// serves all of them and no vector arithmetic competes with LDS.  The results are XOR-
// reduced into ``out`` so that no access can be removed.
#include "gf2_internal.h"

namespace gf2 {
namespace {

constexpr int kProbeUnroll = 64;

__global__ __launch_bounds__(1024) void lds_read_probe(uint64_t* __restrict__ out, int iters) {
  __shared__ uint4 buf[65536 / 16];
  for (int i = threadIdx.x; i < 65536 / 16; i += 1024) buf[i] = make_uint4(i, 3 * i + 1, 5 * i + 2, 7 * i + 3);
  __syncthreads();
  const int L = threadIdx.x & 63;
  uint32_t off = ((uint32_t)((L >> 2) & 3) << 6) | ((uint32_t)(L & 3) << 4);
  uint4 acc = make_uint4(0, 0, 0, 0);
  for (int it = 0; it < iters; ++it) {
    asm volatile("" : "+v"(off));   // the address is opaque to the compiler: no load is hoisted
    const char* base = reinterpret_cast<const char*>(buf) + off;
#pragma unroll
    for (int j = 0; j < kProbeUnroll; ++j) {
      const uint4 v = *reinterpret_cast<const uint4*>(base + ((j * 37) & 255) * 256);
      acc = make_uint4(acc.x ^ v.x, acc.y ^ v.y, acc.z ^ v.z, acc.w ^ v.w);
    }
  }
  out[(size_t)blockIdx.x * 1024 + threadIdx.x] = ((uint64_t)(acc.x ^ acc.y) << 32) | (acc.z ^ acc.w);
}

__global__ __launch_bounds__(1024) void lds_write_probe(uint64_t* __restrict__ out, int iters) {
  __shared__ uint32_t buf[65536 / 4];
  const int L = threadIdx.x & 63;
  uint32_t off = (uint32_t)L * 4u;
  uint32_t v = threadIdx.x;
  for (int it = 0; it < iters; ++it) {
    asm volatile("" : "+v"(off), "+v"(v));
    char* base = reinterpret_cast<char*>(buf) + off;
#pragma unroll
    for (int j = 0; j < kProbeUnroll; ++j) {
      *reinterpret_cast<uint32_t*>(base + ((j * 37) & 255) * 256) = v ^ (uint32_t)j;
    }
  }
  __syncthreads();
  out[(size_t)blockIdx.x * 1024 + threadIdx.x] = buf[(threadIdx.x * 16) & 16383];
}

}  // namespace
}  // namespace gf2

using namespace gf2;

extern "C" gf2_status gf2_lds_probe(int32_t mode, int32_t blocks, int32_t iters, uint64_t* out, double* bytes,
                                    void* stream) {
  if ((mode != 0 && mode != 1) || blocks < 1 || iters < 1 || !out)
    return set_error(GF2_ERR_INVALID_ARG, "gf2_lds_probe: mode 0 or 1, blocks >= 1, iters >= 1, out not NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (mode == 0) hipLaunchKernelGGL(lds_read_probe, dim3(blocks), dim3(1024), 0, s, out, iters);
  else hipLaunchKernelGGL(lds_write_probe, dim3(blocks), dim3(1024), 0, s, out, iters);
  if (bytes) *bytes = (double)blocks * iters * kProbeUnroll * 1024.0 * (mode == 0 ? 16.0 : 4.0);
  return hip_check(hipGetLastError(), "gf2_lds_probe launch");
}
