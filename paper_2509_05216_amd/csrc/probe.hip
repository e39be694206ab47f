// HBM bandwidth probe: a plain grid-stride copy with 16-byte accesses.
//
// It measures the achievable read+write bandwidth of the device (the
// denominator of the stage rooflines) and, having a known byte count, serves as
// the calibration kernel for hardware traffic counters.
#include "internal.h"

namespace isogs {
namespace {

constexpr int kPer = 4;  // 16-byte words per thread, all loads issued before the stores

typedef float f4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_copy16(const f4* __restrict__ src, f4* __restrict__ dst,
                                                size_t n16) {
  const size_t base = (size_t)blockIdx.x * (256 * kPer) + threadIdx.x;
  f4 v[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const size_t i = base + (size_t)k * 256;
    if (i < n16) v[k] = __builtin_nontemporal_load(src + i);
  }
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const size_t i = base + (size_t)k * 256;
    if (i < n16) __builtin_nontemporal_store(v[k], dst + i);
  }
}

}  // namespace

gs_status launch_copy_probe(Ctx* ctx, const void* src, void* dst, size_t bytes, hipStream_t s) {
  (void)ctx;
  const size_t n16 = bytes / 16;
  if (n16 == 0) return GS_OK;
  const size_t blocks = (n16 + 256 * kPer - 1) / (256 * kPer);
  if (blocks > 0x7fffffffULL) {
    set_error("copy probe: %zu bytes is too large", bytes);
    return GS_ERR_INVALID;
  }
  hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, s, (const f4*)src,
                     (f4*)dst, n16);
  GS_LAUNCHED("copy_probe");
  return GS_OK;
}

}  // namespace isogs
