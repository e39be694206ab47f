// Front-to-back alpha compositing of each tile's sorted list (forward) and its
// reverse traversal (backward).
//
// One workgroup per tile, one pixel per thread (TILE x TILE threads: 1, 4 or
// 16 waves).  The tile's records are staged through LDS in batches of DEPTH
// splats (48 B each); every lane of a wave reads the same LDS address, so the
// reads are broadcasts.  The forward stops a batch loop once every pixel of
// the tile has terminated (block-wide vote).
//
// The backward walks the list from the tile's last contributor down to its
// first, recomputing each pixel's transmittance as T / (1 - alpha) from the
// final value, so no per-pixel list is stored.  Per-pair gradients (9 floats)
// are summed over the wave with cross-lane shuffles, combined across the
// workgroup's waves with LDS float atomics, and added to the per-Gaussian
// accumulators with one global atomic per component per (tile, Gaussian).
//
// Both kernels evaluate a pair with the same inline code; the library is
// compiled with -ffp-contract=off, so the forward's skip/stop decisions are
// reproduced exactly by the backward.
#include "internal.h"

namespace isogs {
namespace {

constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;

struct SplatL {
  float A, B, C, o;
  int cx, cy;
  float fx, fy;
  float r, g, b, depth;
};

__device__ inline SplatL to_splat(float4 q0, float4 q1, float4 q2) {
  SplatL s;
  s.A = q0.x; s.B = q0.y; s.C = q0.z; s.o = q0.w;
  s.cx = __float_as_int(q1.x); s.cy = __float_as_int(q1.y);
  s.fx = q1.z; s.fy = q1.w;
  s.r = q2.x; s.g = q2.y; s.b = q2.z; s.depth = q2.w;
  return s;
}

// power = -1/2 (A dx^2 + C dy^2) - B dx dy at pixel (px, py); dx = px + 0.5 - mean_x.
__device__ inline void pair_eval(float A, float B, float C, int cx, int cy, float fx, float fy,
                                 int px, int py, float& dx, float& dy, float& power) {
  dx = (float)(px - cx) + fx;
  dy = (float)(py - cy) + fy;
  power = -0.5f * (A * dx * dx + C * dy * dy) - B * dx * dy;
}

template <int TILE, int DEPTH>
__global__ __launch_bounds__(TILE* TILE) void k_blend_fwd(ViewTable vt,
                                                          const uint2* __restrict__ ranges,
                                                          const uint32_t* __restrict__ tval,
                                                          const float4* __restrict__ splat,
                                                          float* __restrict__ finalT,
                                                          uint32_t* __restrict__ ncon) {
  constexpr int NT = TILE * TILE;
  __shared__ float4 s0[DEPTH], s1[DEPTH], s2[DEPTH];
  const int gt = blockIdx.x;
  const int v = view_of_tile(vt, gt);
  const CamDev& cam = vt.v[v];
  const int lt = gt - cam.tile_offset;
  const int tx = lt % cam.tiles_x, ty = lt / cam.tiles_x;
  const int px = tx * TILE + (int)(threadIdx.x % TILE);
  const int py = ty * TILE + (int)(threadIdx.x / TILE);
  const bool inside = px < cam.W && py < cam.H;
  const uint2 rg = ranges[gt];
  float T = 1.f, cr = 0.f, cg = 0.f, cb = 0.f;
  uint32_t last = 0;
  bool done = !inside;
  for (uint32_t base = rg.x; base < rg.y; base += DEPTH) {
    if (__syncthreads_count(done) == NT) break;
    const int cnt = (int)min((uint32_t)DEPTH, rg.y - base);
    for (int j = threadIdx.x; j < cnt; j += NT) {
      const size_t idx = tval[base + j];
      s0[j] = splat[idx * 3 + 0];
      s1[j] = splat[idx * 3 + 1];
      s2[j] = splat[idx * 3 + 2];
    }
    __syncthreads();
    if (!done) {
      for (int j = 0; j < cnt; ++j) {
        const float4 q0 = s0[j], q1 = s1[j];
        float dx, dy, power;
        pair_eval(q0.x, q0.y, q0.z, __float_as_int(q1.x), __float_as_int(q1.y), q1.z, q1.w, px,
                  py, dx, dy, power);
        if (power > 0.f) continue;
        const float alpha = fminf(kAlphaMax, q0.w * __expf(power));
        if (alpha < kAlphaMin) continue;
        const float Tn = T * (1.f - alpha);
        if (Tn < kTMin) {
          done = true;
          break;
        }
        const float4 q2 = s2[j];
        const float w = alpha * T;
        cr += q2.x * w;
        cg += q2.y * w;
        cb += q2.z * w;
        T = Tn;
        last = base + (uint32_t)j - rg.x + 1u;
      }
    }
  }
  if (inside) {
    const size_t pix = (size_t)py * cam.W + px;
    const size_t plane = (size_t)cam.W * cam.H;
    cam.image[pix] = cr + T * vt.bg[0];
    cam.image[plane + pix] = cg + T * vt.bg[1];
    cam.image[2 * plane + pix] = cb + T * vt.bg[2];
    finalT[cam.pix_offset + pix] = T;
    ncon[cam.pix_offset + pix] = last;
  }
}

__device__ inline float wave_sum(float x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

template <int TILE, int DEPTH>
__global__ __launch_bounds__(TILE* TILE) void k_blend_bwd(ViewTable vt, int n_gauss,
                                                          const uint2* __restrict__ ranges,
                                                          const uint32_t* __restrict__ tval,
                                                          const float4* __restrict__ splat,
                                                          const float* __restrict__ finalT,
                                                          const uint32_t* __restrict__ ncon,
                                                          float* __restrict__ acc) {
  constexpr int NT = TILE * TILE;
  constexpr int NW = NT / 64;
  __shared__ float4 s0[DEPTH], s1[DEPTH], s2[DEPTH];
  __shared__ uint32_t sidx[DEPTH];
  __shared__ float part[DEPTH * 9];
  __shared__ uint32_t smax[NW];
  const int gt = blockIdx.x;
  const int v = view_of_tile(vt, gt);
  const CamDev& cam = vt.v[v];
  const int lt = gt - cam.tile_offset;
  const int tx = lt % cam.tiles_x, ty = lt / cam.tiles_x;
  const int px = tx * TILE + (int)(threadIdx.x % TILE);
  const int py = ty * TILE + (int)(threadIdx.x / TILE);
  const bool inside = px < cam.W && py < cam.H;
  const uint2 rg = ranges[gt];
  const int lane = __lane_id(), wave = threadIdx.x / 64;

  float T = 1.f, dr = 0.f, dg = 0.f, db = 0.f;
  uint32_t nc = 0;
  if (inside) {
    const size_t pix = (size_t)py * cam.W + px;
    const size_t plane = (size_t)cam.W * cam.H;
    T = finalT[cam.pix_offset + pix];
    nc = ncon[cam.pix_offset + pix];
    dr = cam.dimg[pix];
    dg = cam.dimg[plane + pix];
    db = cam.dimg[2 * plane + pix];
  }
  // colour composited behind the current record (starts with T_final * bg)
  float Sr = T * vt.bg[0], Sg = T * vt.bg[1], Sb = T * vt.bg[2];
  // tile-wide last contributor
  uint32_t m = nc;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, d, 64));
  if (lane == 0) smax[wave] = m;
  __syncthreads();
  uint32_t maxn = 0;
  for (int w = 0; w < NW; ++w) maxn = max(maxn, smax[w]);

  for (int hi = (int)maxn; hi > 0; hi -= DEPTH) {
    const int lo = max(0, hi - DEPTH);
    const int cnt = hi - lo;
    __syncthreads();
    for (int j = threadIdx.x; j < cnt; j += NT) {
      const uint32_t idx = tval[rg.x + lo + j];
      sidx[j] = idx;
      s0[j] = splat[(size_t)idx * 3 + 0];
      s1[j] = splat[(size_t)idx * 3 + 1];
      s2[j] = splat[(size_t)idx * 3 + 2];
    }
    for (int j = threadIdx.x; j < cnt * 9; j += NT) part[j] = 0.f;
    __syncthreads();
    for (int j = cnt - 1; j >= 0; --j) {
      const int pos = lo + j;  // position in the tile list
      float g[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) g[k] = 0.f;
      bool contrib = inside && (uint32_t)pos < nc;
      if (contrib) {
        const float4 q0 = s0[j], q1 = s1[j];
        float dx, dy, power;
        pair_eval(q0.x, q0.y, q0.z, __float_as_int(q1.x), __float_as_int(q1.y), q1.z, q1.w, px,
                  py, dx, dy, power);
        const float G = __expf(power);
        const float a_raw = q0.w * G;
        const float alpha = fminf(kAlphaMax, a_raw);
        if (power > 0.f || alpha < kAlphaMin) {
          contrib = false;
        } else {
          const float4 q2 = s2[j];
          const float oma = 1.f - alpha;
          T = T / oma;  // transmittance before this record
          const float w = alpha * T;
          g[6] = w * dr;
          g[7] = w * dg;
          g[8] = w * db;
          const float dalpha = dr * (q2.x * T - Sr / oma) + dg * (q2.y * T - Sg / oma) +
                               db * (q2.z * T - Sb / oma);
          Sr += q2.x * w;
          Sg += q2.y * w;
          Sb += q2.z * w;
          if (a_raw <= kAlphaMax) {
            const float dpow = dalpha * alpha;
            g[5] = dalpha * G;
            g[2] = -0.5f * dpow * dx * dx;
            g[3] = -dpow * dx * dy;
            g[4] = -0.5f * dpow * dy * dy;
            g[0] = dpow * (q0.x * dx + q0.y * dy);
            g[1] = dpow * (q0.y * dx + q0.z * dy);
          }
        }
      }
      if (__any(contrib)) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          const float s = wave_sum(g[k]);
          if (lane == 0 && s != 0.f) atomicAdd(&part[j * 9 + k], s);
        }
      }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < cnt * 9; t += NT) {
      const float s = part[t];
      if (s != 0.f) {
        const int j = t / 9, k = t - j * 9;
        const uint32_t idx = sidx[j];
        const uint32_t vv = idx / (uint32_t)n_gauss, gi = idx - vv * (uint32_t)n_gauss;
        atomicAdd(acc + ((size_t)vv * 9 + k) * n_gauss + gi, s);
      }
    }
  }
}

template <int TILE, int DEPTH>
gs_status fwd_t(const ViewTable& vt, Frame& f, hipStream_t s) {
  hipLaunchKernelGGL((k_blend_fwd<TILE, DEPTH>), dim3(vt.total_tiles), dim3(TILE * TILE), 0, s,
                     vt, (const uint2*)f.ranges.p, (const uint32_t*)f.tval[f.tkey_sel].p,
                     (const float4*)f.splat.p, (float*)f.finalT.p, (uint32_t*)f.ncon.p);
  GS_LAUNCHED("blend_fwd");
  return GS_OK;
}

template <int TILE, int DEPTH>
gs_status bwd_t(const ViewTable& vt, Frame& f, hipStream_t s) {
  hipLaunchKernelGGL((k_blend_bwd<TILE, DEPTH>), dim3(vt.total_tiles), dim3(TILE * TILE), 0, s,
                     vt, (int)f.n, (const uint2*)f.ranges.p,
                     (const uint32_t*)f.tval[f.tkey_sel].p, (const float4*)f.splat.p,
                     (const float*)f.finalT.p, (const uint32_t*)f.ncon.p, (float*)f.acc.p);
  GS_LAUNCHED("blend_bwd");
  return GS_OK;
}

#define GS_DISPATCH(FN, tile, depth, ...)                                   \
  switch (tile * 1000 + depth) {                                            \
    case 8032: return FN<8, 32>(__VA_ARGS__);                               \
    case 8064: return FN<8, 64>(__VA_ARGS__);                               \
    case 16032: return FN<16, 32>(__VA_ARGS__);                             \
    case 16064: return FN<16, 64>(__VA_ARGS__);                             \
    case 16128: return FN<16, 128>(__VA_ARGS__);                            \
    case 16256: return FN<16, 256>(__VA_ARGS__);                            \
    case 32032: return FN<32, 32>(__VA_ARGS__);                             \
    case 32064: return FN<32, 64>(__VA_ARGS__);                             \
    case 32128: return FN<32, 128>(__VA_ARGS__);                            \
    case 32256: return FN<32, 256>(__VA_ARGS__);                            \
    default:                                                                \
      set_error("unsupported tile %d / lds depth %d", tile, depth);         \
      return GS_ERR_UNSUPPORTED;                                            \
  }

}  // namespace

gs_status launch_blend_fwd(const ViewTable& vt, Frame& f, hipStream_t s) {
  GS_DISPATCH(fwd_t, f.tile, f.depth, vt, f, s)
}

gs_status launch_blend_bwd(const ViewTable& vt, Frame& f, hipStream_t s) {
  GS_DISPATCH(bwd_t, f.tile, f.depth, vt, f, s)
}

}  // namespace isogs
