// Adaptive density control of the 3D-GS training that Sec. III adopts by
// citation (clone, split, prune, opacity reset), and the positional-gradient
// statistics that select the Gaussians it acts on.
//
// Statistics: one thread per Gaussian walks the frame's views, reading the
// (view, Gaussian) tile rectangle (touched or not), the kept screen-space mean
// gradient (the first two of the eight geometric sums of the backward) and the
// pixel radius kept by the forward, and updates grad / count / max_radius.
//
// Densification: three launches over blocks of 1024 Gaussians.
//  count  classify every Gaussian (decisions in float64: the mean gradient is
//         the quotient of a float32 sum and an integer count, compared with a
//         float64 threshold, as in any float64 evaluation of the definition);
//         per-block totals of kept originals, clones, split parents with kept
//         children, and splits, from wave ballots;
//  scan   one block turns the block totals into exclusive block offsets and
//         the grand totals (read back by the host to size the output);
//  apply  classify again, rank each Gaussian inside its block in index order
//         (ballot prefix counts), and write every output: originals and clones
//         copy their 11 + 3(d+1)^2 parameter rows (and, for originals, both
//         Adam moments); children get drawn means and reduced log-scales; the
//         moments of new Gaussians are zero.
#include "internal.h"

namespace isogs {
namespace {

constexpr int kDB = 256;        // threads per block
constexpr int kDI = 4;          // Gaussians per thread
constexpr int kDG = kDB * kDI;  // Gaussians per block
constexpr int kDW = kDB / 64;   // waves per block
constexpr uint32_t kKeep = 1u, kClone = 2u, kChild = 4u, kSplit = 8u;

struct DensityCfg {
  const float* grad;
  const int32_t* count;
  const int32_t* maxr;
  const float* ls;     // log-scales [3][n]
  const float* logit;  // opacity logits [n]
  long long n;
  double tau, clone_lim, min_op, max_screen, world_lim, log_div;
  int size_on;
};

// Class bits of Gaussian i (the definition's predicates, in float64).
__device__ inline uint32_t classify(const DensityCfg& c, long long i) {
  const int32_t cnt = c.count[i];
  const double g = cnt > 0 ? (double)c.grad[i] / (double)cnt : 0.0;
  const bool sel = g >= c.tau;
  double smax = 0.0, cmax = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double l = (double)c.ls[(size_t)k * c.n + i];
    smax = fmax(smax, exp(l));
    cmax = fmax(cmax, exp(l - c.log_div));
  }
  const double op = 1.0 / (1.0 + exp(-(double)c.logit[i]));
  const bool low = op < c.min_op;
  const bool clone = sel && smax <= c.clone_lim;
  const bool split = sel && smax > c.clone_lim;
  const bool big_ws = smax > c.world_lim;
  const bool big_vs = (double)c.maxr[i] > c.max_screen;
  uint32_t f = 0;
  if (!split && !low && !(c.size_on && (big_vs || big_ws))) f |= kKeep;
  if (clone && !low && !(c.size_on && big_ws)) f |= kClone;
  if (split) {
    f |= kSplit;
    if (!low && !(c.size_on && cmax > c.world_lim)) f |= kChild;
  }
  return f;
}

__device__ inline uint32_t popc(unsigned long long b) { return (uint32_t)__popcll(b); }

__global__ __launch_bounds__(kDB) void k_density_count(DensityCfg c, uint4* __restrict__ tot) {
  __shared__ uint32_t sh[kDW][4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t a = 0, b = 0, d = 0, e = 0;
  for (int k = 0; k < kDI; ++k) {
    const long long i = (long long)blockIdx.x * kDG + k * kDB + threadIdx.x;
    const uint32_t f = i < c.n ? classify(c, i) : 0u;
    a += popc(__ballot((f & kKeep) != 0));
    b += popc(__ballot((f & kClone) != 0));
    d += popc(__ballot((f & kChild) != 0));
    e += popc(__ballot((f & kSplit) != 0));
  }
  if (lane == 0) {
    sh[w][0] = a;
    sh[w][1] = b;
    sh[w][2] = d;
    sh[w][3] = e;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint4 t = make_uint4(0, 0, 0, 0);
    for (int q = 0; q < kDW; ++q) {
      t.x += sh[q][0];
      t.y += sh[q][1];
      t.z += sh[q][2];
      t.w += sh[q][3];
    }
    tot[blockIdx.x] = t;
  }
}

// One block of 1024 threads: thread t scans a contiguous run of block totals;
// the run sums are scanned in LDS; off[j] = exclusive offsets, off[nb] = totals.
__global__ __launch_bounds__(1024) void k_density_scan(const uint4* __restrict__ tot, int nb,
                                                       uint4* __restrict__ off) {
  __shared__ uint4 run[1024];
  const int t = threadIdx.x;
  const int per = (nb + 1023) / 1024;
  const int lo = min(nb, t * per), hi = min(nb, lo + per);
  uint4 s = make_uint4(0, 0, 0, 0);
  for (int j = lo; j < hi; ++j) {
    const uint4 v = tot[j];
    s.x += v.x;
    s.y += v.y;
    s.z += v.z;
    s.w += v.w;
  }
  run[t] = s;
  __syncthreads();
  for (int st = 1; st < 1024; st <<= 1) {
    uint4 v = make_uint4(0, 0, 0, 0);
    if (t >= st) v = run[t - st];
    __syncthreads();
    if (t >= st) {
      uint4 r = run[t];
      r.x += v.x;
      r.y += v.y;
      r.z += v.z;
      r.w += v.w;
      run[t] = r;
    }
    __syncthreads();
  }
  uint4 base = t > 0 ? run[t - 1] : make_uint4(0, 0, 0, 0);
  for (int j = lo; j < hi; ++j) {
    off[j] = base;
    const uint4 v = tot[j];
    base.x += v.x;
    base.y += v.y;
    base.z += v.z;
    base.w += v.w;
  }
  if (t == 1023) off[nb] = run[1023];
}

// Parameter row r (0..10 + rows of sh) of a SoA set.
__device__ inline float* prow(const gs_params& p, int r) {
  const size_t n = (size_t)p.n;
  if (r < 3) return p.means + (size_t)r * n;
  if (r < 6) return p.log_scales + (size_t)(r - 3) * n;
  if (r < 10) return p.quats + (size_t)(r - 6) * n;
  if (r == 10) return p.opacity_logits;
  return p.sh + (size_t)(r - 11) * n;
}

// Box-Muller in float64 on a Philox pair: u = ((a >> 8) + 0.5) 2^-24,
// theta = 2 pi (b >> 8) 2^-24, (r cos theta, r sin theta), r = sqrt(-2 ln u).
__device__ inline void box_muller64(uint32_t a, uint32_t b, double& z0, double& z1) {
  const double ua = ((double)(a >> 8) + 0.5) * 0x1p-24;
  const double r = sqrt(-2.0 * log(ua));
  const double th = 6.283185307179586 * ((double)(b >> 8) * 0x1p-24);
  z0 = r * cos(th);
  z1 = r * sin(th);
}

struct ApplyArgs {
  gs_params p, m, v;           // inputs (n entries)
  gs_params po, mo, vo;        // outputs (n_out entries)
  int32_t* src;                // optional source index per output
  const uint4* off;            // block offsets; off[nb] = totals
  int nb, rows, n_split;
  uint32_t k0, k1;             // Philox key
};

__global__ __launch_bounds__(kDB) void k_density_apply(DensityCfg c, ApplyArgs a) {
  __shared__ uint32_t sh[kDW][3];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const uint4 tot = a.off[a.nb];
  const uint4 bo = a.off[blockIdx.x];
  uint32_t base0 = bo.x, base1 = bo.y, base2 = bo.z;
  for (int k = 0; k < kDI; ++k) {
    const long long i = (long long)blockIdx.x * kDG + k * kDB + threadIdx.x;
    const uint32_t f = i < c.n ? classify(c, i) : 0u;
    const unsigned long long b0 = __ballot((f & kKeep) != 0);
    const unsigned long long b1 = __ballot((f & kClone) != 0);
    const unsigned long long b2 = __ballot((f & kChild) != 0);
    if (lane == 0) {
      sh[w][0] = popc(b0);
      sh[w][1] = popc(b1);
      sh[w][2] = popc(b2);
    }
    __syncthreads();
    uint32_t p0 = 0, p1 = 0, p2 = 0, t0 = 0, t1 = 0, t2 = 0;
    for (int q = 0; q < kDW; ++q) {
      if (q < w) {
        p0 += sh[q][0];
        p1 += sh[q][1];
        p2 += sh[q][2];
      }
      t0 += sh[q][0];
      t1 += sh[q][1];
      t2 += sh[q][2];
    }
    __syncthreads();
    if (f != 0) {
      const size_t n = (size_t)c.n;
      if (f & kKeep) {
        const size_t o = base0 + p0 + popc(b0 & below);
        for (int r = 0; r < a.rows; ++r) {
          prow(a.po, r)[o] = prow(a.p, r)[i];
          prow(a.mo, r)[o] = prow(a.m, r)[i];
          prow(a.vo, r)[o] = prow(a.v, r)[i];
        }
        if (a.src) a.src[o] = (int32_t)i;
      }
      if (f & kClone) {
        const size_t o = (size_t)tot.x + base1 + p1 + popc(b1 & below);
        for (int r = 0; r < a.rows; ++r) {
          prow(a.po, r)[o] = prow(a.p, r)[i];
          prow(a.mo, r)[o] = 0.f;
          prow(a.vo, r)[o] = 0.f;
        }
        if (a.src) a.src[o] = (int32_t)i;
      }
      if (f & kChild) {
        const size_t o0 = (size_t)tot.x + tot.y +
                          (size_t)a.n_split * (base2 + p2 + popc(b2 & below));
        // parent's rotation R(q / |q|) and scales, in float64
        double q[4];
        for (int r = 0; r < 4; ++r) q[r] = (double)a.p.quats[(size_t)r * n + i];
        const double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        const double qw = q[0] / qn, qx = q[1] / qn, qy = q[2] / qn, qz = q[3] / qn;
        const double R[3][3] = {
            {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy)},
            {2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx)},
            {2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)}};
        double ls[3], s[3], mu[3];
        for (int r = 0; r < 3; ++r) {
          ls[r] = (double)a.p.log_scales[(size_t)r * n + i];
          s[r] = exp(ls[r]);
          mu[r] = (double)a.p.means[(size_t)r * n + i];
        }
        for (int ch = 0; ch < a.n_split; ++ch) {
          const size_t o = o0 + ch;
          uint32_t ctr[4] = {(uint32_t)i, 16u + (uint32_t)ch, 0u, 0u};
          philox4x32_10(ctr, a.k0, a.k1);
          double z[4];
          box_muller64(ctr[0], ctr[1], z[0], z[1]);
          box_muller64(ctr[2], ctr[3], z[2], z[3]);
          const double l0 = s[0] * z[0], l1 = s[1] * z[1], l2 = s[2] * z[2];
          for (int r = 0; r < 3; ++r) {
            prow(a.po, r)[o] = (float)(mu[r] + (R[r][0] * l0 + R[r][1] * l1 + R[r][2] * l2));
            prow(a.po, 3 + r)[o] = (float)(ls[r] - c.log_div);
          }
          for (int r = 6; r < a.rows; ++r) prow(a.po, r)[o] = prow(a.p, r)[i];
          for (int r = 0; r < a.rows; ++r) {
            prow(a.mo, r)[o] = 0.f;
            prow(a.vo, r)[o] = 0.f;
          }
          if (a.src) a.src[o] = (int32_t)i;
        }
      }
    }
    base0 += t0;
    base1 += t1;
    base2 += t2;
  }
}

struct ViewDims {
  float hw[kMaxViews], hh[kMaxViews];  // W/2, H/2 per view
};

__global__ __launch_bounds__(256) void k_density_accumulate(
    const float* __restrict__ accG, const uint2* __restrict__ rect,
    const int32_t* __restrict__ radii, ViewDims vd, int views, long long n, float scale,
    float* __restrict__ grad, int32_t* __restrict__ count, int32_t* __restrict__ maxr) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float g = grad[i];
  int32_t cnt = count[i], mr = maxr[i];
  for (int v = 0; v < views; ++v) {
    const size_t o = (size_t)v * n + i;
    const uint2 r = rect[o];
    if ((r.y & 0xffffu) < (r.x & 0xffffu)) continue;  // touched no tile
    const float2 d = *reinterpret_cast<const float2*>(accG + o * kAccG);
    const float gx = d.x * vd.hw[v], gy = d.y * vd.hh[v];
    g += scale * sqrtf(gx * gx + gy * gy);
    cnt += 1;
    mr = max(mr, radii[o]);
  }
  grad[i] = g;
  count[i] = cnt;
  maxr[i] = mr;
}

__global__ __launch_bounds__(256) void k_opacity_reset(float* __restrict__ logit,
                                                       float* __restrict__ m,
                                                       float* __restrict__ v, long long n,
                                                       double lim) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if ((double)logit[i] > lim) logit[i] = (float)lim;
  m[i] = 0.f;
  v[i] = 0.f;
}

}  // namespace

gs_status launch_density_accumulate(const Frame& f, const gs_density_stats& st, float scale,
                                    hipStream_t s) {
  if (f.n == 0) return GS_OK;
  ViewDims vd;
  for (int v = 0; v < f.views; ++v) {
    vd.hw[v] = 0.5f * (float)f.vt.v[v].W;
    vd.hh[v] = 0.5f * (float)f.vt.v[v].H;
  }
  hipLaunchKernelGGL(k_density_accumulate, dim3((unsigned)((f.n + 255) / 256)), dim3(256), 0, s,
                     (const float*)f.acc.p, (const uint2*)f.rect.p, (const int32_t*)f.radii.p,
                     vd, f.views, (long long)f.n, scale, st.grad, st.count, st.max_radius);
  GS_LAUNCHED("density_accumulate");
  return GS_OK;
}

gs_status densify_run(Ctx* ctx, const gs_params& p, const gs_params& m, const gs_params& v,
                      const gs_density_stats& st, const gs_density_opts& o, const gs_params* p_out,
                      const gs_params* m_out, const gs_params* v_out, int32_t* src_index,
                      gs_density_info* info, hipStream_t s) {
  const long long n = p.n;
  const int nb = (int)((n + kDG - 1) / kDG);
  DensityCfg c;
  c.grad = st.grad;
  c.count = st.count;
  c.maxr = st.max_radius;
  c.ls = p.log_scales;
  c.logit = p.opacity_logits;
  c.n = n;
  c.tau = o.grad_threshold;
  c.clone_lim = o.percent_dense * o.extent;
  c.min_op = o.min_opacity;
  c.max_screen = o.max_screen;
  c.world_lim = o.max_world * o.extent;
  c.log_div = std::log(o.split_div);
  c.size_on = o.max_screen > 0.0 ? 1 : 0;
  // block totals [nb], offsets [nb + 1]
  const size_t bytes = sizeof(uint4) * (2 * (size_t)nb + 1);
  gs_status stt = buf_ensure(ctx, ctx->dens_blk, bytes, s);
  if (stt != GS_OK) return stt;
  if (ctx->dens_host == nullptr)
    GS_HIP(hipHostMalloc((void**)&ctx->dens_host, sizeof(uint4), hipHostMallocDefault));
  uint4* tot = (uint4*)ctx->dens_blk.p;
  uint4* off = tot + nb;
  if (nb > 0) {
    hipLaunchKernelGGL(k_density_count, dim3(nb), dim3(kDB), 0, s, c, tot);
    GS_LAUNCHED("density_count");
  }
  hipLaunchKernelGGL(k_density_scan, dim3(1), dim3(1024), 0, s, (const uint4*)tot, nb, off);
  GS_LAUNCHED("density_scan");
  GS_HIP(hipMemcpyAsync(ctx->dens_host, off + nb, sizeof(uint4), hipMemcpyDeviceToHost, s));
  GS_HIP(hipStreamSynchronize(s));
  const uint4 t = *(const uint4*)ctx->dens_host;
  info->n_in = n;
  info->kept = t.x;
  info->cloned = t.y;
  info->split = t.w;
  info->children = (int64_t)t.z * o.n_split;
  info->n_out = (int64_t)t.x + t.y + info->children;
  info->pruned = n - (int64_t)t.x - t.w;
  if (p_out == nullptr) return GS_OK;
  if (p_out->n < info->n_out || m_out->n < info->n_out || v_out->n < info->n_out) {
    set_error("gs_densify: output sets hold %lld entries; the densified set has %lld",
              (long long)p_out->n, (long long)info->n_out);
    return GS_ERR_CAPACITY;
  }
  if (p_out->n != info->n_out || m_out->n != info->n_out || v_out->n != info->n_out) {
    set_error("gs_densify: output sets must hold exactly %lld entries (p_out.n = %lld)",
              (long long)info->n_out, (long long)p_out->n);
    return GS_ERR_INVALID;
  }
  if (nb == 0) return GS_OK;
  ApplyArgs a;
  a.p = p;
  a.m = m;
  a.v = v;
  a.po = *p_out;
  a.mo = *m_out;
  a.vo = *v_out;
  a.src = src_index;
  a.off = off;
  a.nb = nb;
  a.rows = 11 + (p.sh_degree + 1) * (p.sh_degree + 1) * 3;
  a.n_split = o.n_split;
  a.k0 = (uint32_t)o.seed;
  a.k1 = (uint32_t)(o.seed >> 32);
  hipLaunchKernelGGL(k_density_apply, dim3(nb), dim3(kDB), 0, s, c, a);
  GS_LAUNCHED("density_apply");
  return GS_OK;
}

gs_status launch_opacity_reset(const gs_params& p, const gs_params& m, const gs_params& v,
                               double max_opacity, hipStream_t s) {
  if (p.n == 0) return GS_OK;
  const double lim = std::log(max_opacity / (1.0 - max_opacity));
  hipLaunchKernelGGL(k_opacity_reset, dim3((unsigned)((p.n + 255) / 256)), dim3(256), 0, s,
                     p.opacity_logits, m.opacity_logits, v.opacity_logits, (long long)p.n, lim);
  GS_LAUNCHED("opacity_reset");
  return GS_OK;
}

}  // namespace isogs
