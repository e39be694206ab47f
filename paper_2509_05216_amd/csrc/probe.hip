// HBM bandwidth probe: a plain grid-stride copy with 16-byte accesses.
//
// It measures the achievable read+write bandwidth of the device (the
// denominator of the stage rooflines) and, having a known byte count, serves as
// the calibration kernel for hardware traffic counters.
#include "internal.h"

namespace isogs {
namespace {

__global__ __launch_bounds__(256) void k_copy16(const float4* __restrict__ src,
                                                float4* __restrict__ dst, size_t n16) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n16; i += stride)
    dst[i] = src[i];
}

}  // namespace

gs_status launch_copy_probe(Ctx* ctx, const void* src, void* dst, size_t bytes, hipStream_t s) {
  const size_t n16 = bytes / 16;
  if (n16 == 0) return GS_OK;
  // enough waves to cover every CU several times over, no more than the data needs
  size_t blocks = (size_t)ctx->cu_count * 16;
  const size_t need = (n16 + 255) / 256;
  if (blocks > need) blocks = need;
  hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, s, (const float4*)src,
                     (float4*)dst, n16);
  GS_LAUNCHED("copy_probe");
  return GS_OK;
}

}  // namespace isogs
