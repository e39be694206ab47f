// Isosurface points and ray-cast target views of a device-resident volume: the
// extraction and rendering that Sec. III does with ParaView, done on the GPU so
// a volume already in HBM (the in-situ setting of Sec. V) never leaves it.
//
// Extraction: edge crossings of the iso level (the vertex rule of marching
// cubes) in a canonical order: vertices row-major (k, j, i), per vertex its
// +x, +y, +z edges.  Three launches over blocks of 4096 vertices (16 per
// thread, lanes on consecutive i so the value loads are coalesced; the +y and
// +z neighbours come through L2): count per block (three ballots per vertex
// group), scan (one block), emit (the same predicates, ranked inside the block
// by ballot prefix counts, points written in order).  A crossing on edge e
// is kept when the Philox4x32-10 uniform of counter (e lo, e hi, 3, 0) is
// below keep_prob, so a subsample needs no sort and is the same however the
// grid is blocked.  Positions and the interpolation parameter in float64.
//
// Ray-cast: one thread per pixel, all arithmetic in float64 (the FP64 vector
// rate equals the non-packed FP32 rate here, and float64 keeps the marching
// and bisection decisions those of any float64 evaluation): slab clipping to
// the box, samples at t_near + k step of the trilinear interpolant, the first
// rise through iso, ten bisections, headlight shading with the interpolant's
// gradient.
#include "internal.h"

namespace isogs {
namespace {

constexpr int kIB = 256;          // threads per block
constexpr int kIV = 16;           // vertices per thread
constexpr int kIG = kIB * kIV;    // vertices per block
constexpr int kIW = kIB / 64;

struct VolDev {
  const float* v;
  long long nx, ny, nz;
  double lo[3], h[3];
  float iso;
};

struct KeepRule {
  uint32_t k0, k1;
  float prob;  // >= 1: keep all
};

__device__ inline bool kept(const KeepRule& r, unsigned long long e) {
  if (r.prob >= 1.0f) return true;
  uint32_t c[4] = {(uint32_t)e, (uint32_t)(e >> 32), 3u, 0u};
  philox4x32_10(c, r.k0, r.k1);
  return (float)(c[0] >> 8) * (1.0f / 16777216.0f) < r.prob;
}

// Crossing flags of vertex `vid` (bit a: its edge along axis a crosses and is
// kept) and the values at the vertex (v0) and its +x, +y, +z neighbours.  The
// strict sign tests compare the float32 values with iso directly (exact).
__device__ inline bool crosses(float a, float b, float iso) {
  return (a < iso && b > iso) || (a > iso && b < iso);
}

__device__ inline uint32_t edge_flags(const VolDev& V, const KeepRule& r, long long vid,
                                      long long nvert, float& v0, float& v1, float& v2,
                                      float& v3) {
  if (vid >= nvert) return 0u;
  const long long i = vid % V.nx;
  const long long jk = vid / V.nx;
  const long long j = jk % V.ny;
  const long long k = jk / V.ny;
  v0 = V.v[vid];
  uint32_t f = 0;
  const unsigned long long e = 3ull * (unsigned long long)vid;
  if (i + 1 < V.nx) {
    v1 = V.v[vid + 1];
    if (crosses(v0, v1, V.iso) && kept(r, e)) f |= 1u;
  }
  if (j + 1 < V.ny) {
    v2 = V.v[vid + V.nx];
    if (crosses(v0, v2, V.iso) && kept(r, e + 1)) f |= 2u;
  }
  if (k + 1 < V.nz) {
    v3 = V.v[vid + V.nx * V.ny];
    if (crosses(v0, v3, V.iso) && kept(r, e + 2)) f |= 4u;
  }
  return f;
}

__device__ inline uint32_t popc(unsigned long long b) { return (uint32_t)__popcll(b); }

__global__ __launch_bounds__(kIB) void k_iso_count(VolDev V, KeepRule r, long long nvert,
                                                    uint32_t* __restrict__ tot) {
  __shared__ uint32_t sh[kIW];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t c = 0;
  for (int q = 0; q < kIV; ++q) {
    const long long vid = (long long)blockIdx.x * kIG + q * kIB + threadIdx.x;
    float v0 = 0.f, v1 = 0.f, v2 = 0.f, v3 = 0.f;
    const uint32_t f = edge_flags(V, r, vid, nvert, v0, v1, v2, v3);
    c += popc(__ballot((f & 1u) != 0)) + popc(__ballot((f & 2u) != 0)) +
         popc(__ballot((f & 4u) != 0));
  }
  if (lane == 0) sh[w] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int q = 0; q < kIW; ++q) t += sh[q];
    tot[blockIdx.x] = t;
  }
}

// One block of 1024 threads: exclusive offsets of the block totals (64-bit) and
// the grand total at off[nb].
__global__ __launch_bounds__(1024) void k_iso_scan(const uint32_t* __restrict__ tot, long long nb,
                                                   unsigned long long* __restrict__ off) {
  __shared__ unsigned long long run[1024];
  const int t = threadIdx.x;
  const long long per = (nb + 1023) / 1024;
  const long long lo = min(nb, t * per), hi = min(nb, lo + per);
  unsigned long long s = 0;
  for (long long j = lo; j < hi; ++j) s += tot[j];
  run[t] = s;
  __syncthreads();
  for (int st = 1; st < 1024; st <<= 1) {
    unsigned long long v = 0;
    if (t >= st) v = run[t - st];
    __syncthreads();
    if (t >= st) run[t] += v;
    __syncthreads();
  }
  unsigned long long base = t > 0 ? run[t - 1] : 0ull;
  for (long long j = lo; j < hi; ++j) {
    off[j] = base;
    base += tot[j];
  }
  if (t == 1023) off[nb] = run[1023];
}

__global__ __launch_bounds__(kIB) void k_iso_emit(VolDev V, KeepRule r, long long nvert,
                                                   const unsigned long long* __restrict__ off,
                                                   float* __restrict__ xyz, long long cap) {
  __shared__ uint32_t sh[kIW];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  unsigned long long base = off[blockIdx.x];
  for (int q = 0; q < kIV; ++q) {
    const long long vid = (long long)blockIdx.x * kIG + q * kIB + threadIdx.x;
    float v0 = 0.f, v1 = 0.f, v2 = 0.f, v3 = 0.f;
    const uint32_t f = edge_flags(V, r, vid, nvert, v0, v1, v2, v3);
    const unsigned long long bx = __ballot((f & 1u) != 0);
    const unsigned long long by = __ballot((f & 2u) != 0);
    const unsigned long long bz = __ballot((f & 4u) != 0);
    const uint32_t mine = popc(bx & below) + popc(by & below) + popc(bz & below);
    if (lane == 0) sh[w] = popc(bx) + popc(by) + popc(bz);
    __syncthreads();
    uint32_t pre = 0, all = 0;
    for (int q2 = 0; q2 < kIW; ++q2) {
      if (q2 < w) pre += sh[q2];
      all += sh[q2];
    }
    __syncthreads();
    if (f != 0) {
      const long long i = vid % V.nx;
      const long long jk = vid / V.nx;
      const long long j = jk % V.ny;
      const long long k = jk / V.ny;
      const double px = V.lo[0] + (double)i * V.h[0];
      const double py = V.lo[1] + (double)j * V.h[1];
      const double pz = V.lo[2] + (double)k * V.h[2];
      unsigned long long o = base + pre + mine;
      // t = a / (a - b), a = v0 - iso, b = v1 - iso (both exact in float64)
      const double a = (double)v0 - (double)V.iso;
      if (f & 1u) {
        if ((long long)o < cap) {
          const double t = a / ((double)v0 - (double)v1);
          xyz[o] = (float)(px + t * V.h[0]);
          xyz[cap + o] = (float)py;
          xyz[2 * cap + o] = (float)pz;
        }
        ++o;
      }
      if (f & 2u) {
        if ((long long)o < cap) {
          const double t = a / ((double)v0 - (double)v2);
          xyz[o] = (float)px;
          xyz[cap + o] = (float)(py + t * V.h[1]);
          xyz[2 * cap + o] = (float)pz;
        }
        ++o;
      }
      if (f & 4u) {
        if ((long long)o < cap) {
          const double t = a / ((double)v0 - (double)v3);
          xyz[o] = (float)px;
          xyz[cap + o] = (float)py;
          xyz[2 * cap + o] = (float)(pz + t * V.h[2]);
        }
      }
    }
    base += all;
  }
}

// ------------------------------------------------------------------ ray-cast
struct RayView {
  double R[9], o[3];
  double fx, fy, cx, cy;
  int W, H;
  float* img;
};

struct RayViews {
  RayView v[kMaxViews];
  int n;
};

// Trilinear value (and optionally gradient) of the volume at p.
__device__ inline double trilerp(const VolDev& V, const double* p, double* g) {
  double u[3];
  long long i0[3];
  double fr[3];
  const long long n[3] = {V.nx, V.ny, V.nz};
  for (int a = 0; a < 3; ++a) {
    u[a] = (p[a] - V.lo[a]) / V.h[a];
    long long i = (long long)floor(u[a]);
    i = i < 0 ? 0 : (i > n[a] - 2 ? n[a] - 2 : i);
    i0[a] = i;
    fr[a] = u[a] - (double)i;
  }
  const float* b = V.v + (i0[2] * V.ny + i0[1]) * V.nx + i0[0];
  const long long sy = V.nx, sz = V.nx * V.ny;
  const double c000 = b[0], c100 = b[1], c010 = b[sy], c110 = b[sy + 1];
  const double c001 = b[sz], c101 = b[sz + 1], c011 = b[sz + sy], c111 = b[sz + sy + 1];
  const double fx = fr[0], fy = fr[1], fz = fr[2];
  const double c00 = c000 + fx * (c100 - c000);
  const double c10 = c010 + fx * (c110 - c010);
  const double c01 = c001 + fx * (c101 - c001);
  const double c11 = c011 + fx * (c111 - c011);
  const double c0 = c00 + fy * (c10 - c00);
  const double c1 = c01 + fy * (c11 - c01);
  if (g != nullptr) {
    const double dx0 = (c100 - c000) * (1 - fy) + (c110 - c010) * fy;
    const double dx1 = (c101 - c001) * (1 - fy) + (c111 - c011) * fy;
    g[0] = (dx0 * (1 - fz) + dx1 * fz) / V.h[0];
    g[1] = ((c10 - c00) * (1 - fz) + (c11 - c01) * fz) / V.h[1];
    g[2] = (c1 - c0) / V.h[2];
  }
  return c0 + fz * (c1 - c0);
}

__global__ __launch_bounds__(256) void k_raycast(VolDev V, RayViews rv, double step,
                                                 double hi0, double hi1, double hi2) {
  const RayView& c = rv.v[blockIdx.y];
  const int pix = blockIdx.x * blockDim.x + threadIdx.x;
  if (pix >= c.W * c.H) return;
  const int x = pix % c.W, y = pix / c.W;
  const double dc[3] = {((double)x + 0.5 - c.cx) / c.fx, ((double)y + 0.5 - c.cy) / c.fy, 1.0};
  double d[3];
  for (int a = 0; a < 3; ++a) d[a] = dc[0] * c.R[0 * 3 + a] + dc[1] * c.R[1 * 3 + a] + dc[2] * c.R[2 * 3 + a];
  const double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  for (int a = 0; a < 3; ++a) d[a] /= dn;
  const double hi[3] = {hi0, hi1, hi2};
  double tn = 0.0, tf = INFINITY;
  bool box = true;
  for (int a = 0; a < 3; ++a) {
    if (d[a] == 0.0) {
      if (c.o[a] < V.lo[a] || c.o[a] > hi[a]) box = false;
      continue;
    }
    const double t0 = (V.lo[a] - c.o[a]) / d[a], t1 = (hi[a] - c.o[a]) / d[a];
    tn = fmax(tn, fmin(t0, t1));
    tf = fmin(tf, fmax(t0, t1));
  }
  float rgb[3] = {0.f, 0.f, 0.f};
  if (box && tf > tn) {
    double p[3];
    for (int a = 0; a < 3; ++a) p[a] = c.o[a] + tn * d[a];
    double f_prev = trilerp(V, p, nullptr) - (double)V.iso;
    double lo_t = 0.0, hi_t = -1.0;
    for (long long k = 1;; ++k) {
      const double tk = tn + (double)k * step;
      if (tk > tf) break;
      for (int a = 0; a < 3; ++a) p[a] = c.o[a] + tk * d[a];
      const double f = trilerp(V, p, nullptr) - (double)V.iso;
      if (f_prev < 0.0 && f >= 0.0) {
        lo_t = tn + (double)(k - 1) * step;
        hi_t = tk;
        break;
      }
      f_prev = f;
    }
    if (hi_t >= 0.0) {
      for (int it = 0; it < 10; ++it) {
        const double mid = 0.5 * (lo_t + hi_t);
        for (int a = 0; a < 3; ++a) p[a] = c.o[a] + mid * d[a];
        if (trilerp(V, p, nullptr) - (double)V.iso < 0.0)
          lo_t = mid;
        else
          hi_t = mid;
      }
      const double th = 0.5 * (lo_t + hi_t);
      for (int a = 0; a < 3; ++a) p[a] = c.o[a] + th * d[a];
      double g[3];
      (void)trilerp(V, p, g);
      const double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
      const double lam = gn > 0.0 ? fabs((g[0] * d[0] + g[1] * d[1] + g[2] * d[2]) / gn) : 0.0;
      const double sh = 0.2 + 0.8 * lam;
      rgb[0] = (float)(0.85 * sh);
      rgb[1] = (float)((0.45 + 0.25 * p[2]) * sh);
      rgb[2] = (float)((0.30 + 0.25 * (p[0] + 1.0)) * sh);
    }
  }
  const size_t plane = (size_t)c.W * c.H;
  for (int ch = 0; ch < 3; ++ch) c.img[ch * plane + pix] = rgb[ch];
}

VolDev vol_dev(const gs_volume& vol, float iso) {
  VolDev V;
  V.v = vol.values;
  V.nx = vol.nx;
  V.ny = vol.ny;
  V.nz = vol.nz;
  const long long n[3] = {vol.nx, vol.ny, vol.nz};
  for (int a = 0; a < 3; ++a) {
    V.lo[a] = (double)vol.lo[a];
    V.h[a] = ((double)vol.hi[a] - (double)vol.lo[a]) / (double)(n[a] - 1);
  }
  V.iso = iso;
  return V;
}

}  // namespace

gs_status iso_extract_run(Ctx* ctx, const gs_volume& vol, float iso, float keep_prob,
                          uint64_t seed, float* xyz, int64_t cap, int64_t* n_kept,
                          hipStream_t s) {
  const VolDev V = vol_dev(vol, iso);
  const long long nvert = (long long)vol.nx * vol.ny * vol.nz;
  const long long nb = (nvert + kIG - 1) / kIG;
  KeepRule r{(uint32_t)seed, (uint32_t)(seed >> 32), keep_prob};
  const size_t bytes = sizeof(uint32_t) * (size_t)nb + sizeof(unsigned long long) * (nb + 1);
  gs_status st = buf_ensure(ctx, ctx->iso_blk, bytes, s);
  if (st != GS_OK) return st;
  if (ctx->iso_host == nullptr)
    GS_HIP(hipHostMalloc((void**)&ctx->iso_host, sizeof(unsigned long long),
                         hipHostMallocDefault));
  auto* off = (unsigned long long*)ctx->iso_blk.p;
  auto* tot = (uint32_t*)(off + nb + 1);
  hipLaunchKernelGGL(k_iso_count, dim3((unsigned)nb), dim3(kIB), 0, s, V, r, nvert, tot);
  GS_LAUNCHED("iso_count");
  hipLaunchKernelGGL(k_iso_scan, dim3(1), dim3(1024), 0, s, (const uint32_t*)tot, nb, off);
  GS_LAUNCHED("iso_scan");
  GS_HIP(hipMemcpyAsync(ctx->iso_host, off + nb, sizeof(unsigned long long),
                        hipMemcpyDeviceToHost, s));
  GS_HIP(hipStreamSynchronize(s));
  *n_kept = (int64_t)*ctx->iso_host;
  if (xyz == nullptr) return GS_OK;
  if (*n_kept > cap) {
    set_error("gs_iso_extract: %lld points do not fit the capacity of %lld",
              (long long)*n_kept, (long long)cap);
    return GS_ERR_CAPACITY;
  }
  hipLaunchKernelGGL(k_iso_emit, dim3((unsigned)nb), dim3(kIB), 0, s, V, r, nvert,
                     (const unsigned long long*)off, xyz, (long long)cap);
  GS_LAUNCHED("iso_emit");
  return GS_OK;
}

gs_status launch_raycast(const gs_volume& vol, float iso, const gs_camera* cams, int nv,
                         float* const* images, double step, hipStream_t s) {
  const VolDev V = vol_dev(vol, iso);
  RayViews rv;
  rv.n = nv;
  int max_pix = 0;
  for (int k = 0; k < nv; ++k) {
    RayView& r = rv.v[k];
    const gs_camera& c = cams[k];
    for (int i = 0; i < 9; ++i) r.R[i] = (double)c.R[i];
    // camera centre -R^T t
    for (int a = 0; a < 3; ++a)
      r.o[a] = -((double)c.R[0 * 3 + a] * c.t[0] + (double)c.R[1 * 3 + a] * c.t[1] +
                 (double)c.R[2 * 3 + a] * c.t[2]);
    r.fx = c.fx;
    r.fy = c.fy;
    r.cx = c.cx;
    r.cy = c.cy;
    r.W = c.width;
    r.H = c.height;
    r.img = images[k];
    if (c.width * c.height > max_pix) max_pix = c.width * c.height;
  }
  const dim3 grid((unsigned)((max_pix + 255) / 256), (unsigned)nv);
  hipLaunchKernelGGL(k_raycast, grid, dim3(256), 0, s, V, rv, step, (double)vol.hi[0],
                     (double)vol.hi[1], (double)vol.hi[2]);
  GS_LAUNCHED("raycast");
  return GS_OK;
}

}  // namespace isogs
