// Fused, bias-corrected Adam over every parameter group in one launch.
//
// The groups (means, log-scales, quaternions, opacity logits, SH DC rows, SH
// remaining rows) are contiguous float32 segments with their own learning
// rate.  Blocks are assigned to segments by a prefix table in the kernel
// arguments; each thread updates four consecutive floats with 16-byte loads
// and stores when the segment is 16-byte aligned.  Traffic is 28 bytes per
// parameter: p, g, m, v read, p, m, v written (plus g cleared on request).
#include "internal.h"

namespace isogs {
namespace {

constexpr int kSeg = 6;
constexpr int kThreads = 256;
constexpr int kPerBlock = kThreads * 4;

struct AdamSegs {
  float* p[kSeg];
  float* g[kSeg];
  float* m[kSeg];
  float* v[kSeg];
  long long count[kSeg];
  float lr[kSeg];
  unsigned block_start[kSeg + 1];
  int nseg;
  float b1, b2, eps, inv_bc1, inv_sqrt_bc2;
  int zero_grads;
  const float* dev_bc;    // optional: bias corrections read from the device (graph steps)
  const uint32_t* skip;   // optional: no update while *skip != 0 (record overflow)
};

__device__ inline void adam1(float& p, float& g, float& m, float& v, float lr, float inv_bc1,
                             float inv_sqrt_bc2, const AdamSegs& a) {
  m = a.b1 * m + (1.f - a.b1) * g;
  v = a.b2 * v + (1.f - a.b2) * g * g;
  const float mh = m * inv_bc1;
  const float denom = sqrtf(v) * inv_sqrt_bc2 + a.eps;
  p -= lr * mh / denom;
  if (a.zero_grads) g = 0.f;
}

__global__ __launch_bounds__(kThreads) void k_adam(AdamSegs a) {
  if (a.skip != nullptr && *a.skip != 0u) return;
  const float inv_bc1 = a.dev_bc != nullptr ? a.dev_bc[0] : a.inv_bc1;
  const float inv_sqrt_bc2 = a.dev_bc != nullptr ? a.dev_bc[1] : a.inv_sqrt_bc2;
  int s = 0;
  while (s + 1 < a.nseg && blockIdx.x >= a.block_start[s + 1]) ++s;
  const long long first = ((long long)(blockIdx.x - a.block_start[s]) * kPerBlock) + threadIdx.x * 4;
  const long long n = a.count[s];
  if (first >= n) return;
  float* P = a.p[s];
  float* G = a.g[s];
  float* M = a.m[s];
  float* V = a.v[s];
  const float lr = a.lr[s];
  const bool aligned = ((((uintptr_t)P) | ((uintptr_t)G) | ((uintptr_t)M) | ((uintptr_t)V)) & 15u) == 0;
  if (aligned && first + 4 <= n) {
    float4 p = *(float4*)(P + first), g = *(float4*)(G + first);
    float4 m = *(float4*)(M + first), v = *(float4*)(V + first);
    adam1(p.x, g.x, m.x, v.x, lr, inv_bc1, inv_sqrt_bc2, a);
    adam1(p.y, g.y, m.y, v.y, lr, inv_bc1, inv_sqrt_bc2, a);
    adam1(p.z, g.z, m.z, v.z, lr, inv_bc1, inv_sqrt_bc2, a);
    adam1(p.w, g.w, m.w, v.w, lr, inv_bc1, inv_sqrt_bc2, a);
    *(float4*)(P + first) = p;
    *(float4*)(M + first) = m;
    *(float4*)(V + first) = v;
    if (a.zero_grads) *(float4*)(G + first) = g;
  } else {
    for (long long i = first; i < n && i < first + 4; ++i) {
      float p = P[i], g = G[i], m = M[i], v = V[i];
      adam1(p, g, m, v, lr, inv_bc1, inv_sqrt_bc2, a);
      P[i] = p;
      M[i] = m;
      V[i] = v;
      if (a.zero_grads) G[i] = g;
    }
  }
}

}  // namespace

gs_status launch_adam(const gs_params& p, const gs_params& g, const gs_params& m,
                      const gs_params& v, const gs_adam_opts& o, int64_t step, hipStream_t s,
                      const float* dev_bc, const uint32_t* skip) {
  const long long n = p.n;
  const int nb = (p.sh_degree + 1) * (p.sh_degree + 1);
  AdamSegs a;
  std::memset(&a, 0, sizeof(a));
  struct Src {
    float* pp; float* gg; float* mm; float* vv; long long cnt; float lr;
  } segs[kSeg] = {
      {p.means, g.means, m.means, v.means, 3 * n, o.lr_means},
      {p.log_scales, g.log_scales, m.log_scales, v.log_scales, 3 * n, o.lr_log_scales},
      {p.quats, g.quats, m.quats, v.quats, 4 * n, o.lr_quats},
      {p.opacity_logits, g.opacity_logits, m.opacity_logits, v.opacity_logits, n, o.lr_opacity},
      {p.sh, g.sh, m.sh, v.sh, 3 * n, o.lr_sh_dc},
      {p.sh + 3 * n, g.sh + 3 * n, m.sh + 3 * n, v.sh + 3 * n, (long long)(nb - 1) * 3 * n,
       o.lr_sh_rest},
  };
  unsigned blocks = 0;
  int ns = 0;
  for (int i = 0; i < kSeg; ++i) {
    if (segs[i].cnt <= 0) continue;
    a.p[ns] = segs[i].pp;
    a.g[ns] = segs[i].gg;
    a.m[ns] = segs[i].mm;
    a.v[ns] = segs[i].vv;
    a.count[ns] = segs[i].cnt;
    a.lr[ns] = segs[i].lr;
    a.block_start[ns] = blocks;
    blocks += (unsigned)((segs[i].cnt + kPerBlock - 1) / kPerBlock);
    ++ns;
  }
  a.block_start[ns] = blocks;
  a.nseg = ns;
  a.b1 = o.beta1;
  a.b2 = o.beta2;
  a.eps = o.eps;
  a.inv_bc1 = (float)(1.0 / (1.0 - pow((double)o.beta1, (double)step)));
  a.inv_sqrt_bc2 = (float)(1.0 / sqrt(1.0 - pow((double)o.beta2, (double)step)));
  a.zero_grads = o.zero_grads;
  a.dev_bc = dev_bc;
  a.skip = skip;
  hipLaunchKernelGGL(k_adam, dim3(blocks), dim3(kThreads), 0, s, a);
  GS_LAUNCHED("adam");
  return GS_OK;
}

}  // namespace isogs
