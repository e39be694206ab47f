// Training loss: mean over views of (1 - lambda) L1 + lambda (1 - SSIM), and its
// gradient with respect to the rendered image.
//
// SSIM uses an 11 x 11 Gaussian window (sigma 1.5, separable, weights summing
// to one), C1 = 0.01^2, C2 = 0.03^2, zero padding, averaged over pixels and
// channels.  Two LDS-tiled passes per view and channel (32 x 32 output pixels
// per 256-thread block, a 42 x 42 halo tile): the first forms the five local
// moments by separable filtering and writes, per pixel, the partials
// g1 = dS/dmu_x, g2 = dS/dE[x^2] and g3 = dS/dE[xy]; the second filters those
// maps (the window is symmetric, so the zero-padded correlation is its own
// adjoint) and combines them with the L1 term:
//   dL/dx = s [(1 - lambda) sign(x - y) - lambda (w*g1 + 2 x w*g2 + y w*g3)],
//   s = 1/(3 H W V).
// Horizontal taps share w x between the moments and use explicit fused
// multiply-adds; in the vertical pass each thread produces four consecutive
// rows of one column from 14 LDS rows.  Loss sums are reduced per block into
// float64 partials and summed by a final single-block kernel, so the loss
// value is deterministic.
#include "internal.h"

namespace isogs {
namespace {

constexpr int kT = 32;           // output tile side
constexpr int kR = 5;            // window radius
constexpr int kN = 2 * kR + 1;   // taps
constexpr int kH = kT + 2 * kR;  // 42: halo tile side
constexpr int kP = kH + 1;       // padded LDS row of the halo tile
constexpr int kQ = kT + 1;       // padded LDS row of the horizontal pass
constexpr int kRows = 4;         // output rows per thread in the vertical pass
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;

struct Win {
  float w[kN];
};

constexpr int kLoads = (kH * kH + 255) / 256;  // halo elements per thread

// Halo element t of the tile whose top-left halo pixel is (ox, oy): whether it
// lies in the image, and an in-image offset to read (clamped, so every load is
// valid; the value is replaced by zero padding when outside).
__device__ inline bool halo_inside(int t, int ox, int oy, int W, int H) {
  const int gx = ox + t % kH, gy = oy + t / kH;
  return gx >= 0 && gx < W && gy >= 0 && gy < H;
}

__device__ inline size_t halo_offset(int t, int ox, int oy, int W, int H) {
  const int gx = min(max(ox + t % kH, 0), W - 1), gy = min(max(oy + t / kH, 0), H - 1);
  return (size_t)gy * W + gx;
}

// Thread layout of the vertical pass: column c, rows r0 .. r0 + 3.
__device__ inline void vert_slot(int& c, int& r0) {
  c = threadIdx.x % kT;
  r0 = (threadIdx.x / kT) * kRows;
}

// Vertical filtering of NM moment maps held in LDS (hq[m][row][col]) for the
// four rows of this thread: out[o][m] = sum_i w[i] hq[m][r0 + o + i][c].
template <int NM>
__device__ inline void vert_filter(const float (*hq)[kH][kQ], const Win& win, int c, int r0,
                                   float (*out)[NM]) {
#pragma unroll
  for (int o = 0; o < kRows; ++o)
#pragma unroll
    for (int m = 0; m < NM; ++m) out[o][m] = 0.f;
#pragma unroll
  for (int i = 0; i < kN + kRows - 1; ++i) {
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      const float v = hq[m][r0 + i][c];
#pragma unroll
      for (int o = 0; o < kRows; ++o)
        if (i - o >= 0 && i - o < kN) out[o][m] = fmaf(win.w[i - o], v, out[o][m]);
    }
  }
}

__global__ __launch_bounds__(256) void k_ssim_fwd(const float* __restrict__ x,
                                                  const float* __restrict__ y, int W, int H,
                                                  Win win, float* __restrict__ gmap,
                                                  double* __restrict__ part) {
  __shared__ float sx[kH][kP], sy[kH][kP];
  __shared__ float hq[5][kH][kQ];
  const int ch = blockIdx.z;
  const size_t plane = (size_t)W * H;
  const float* xc = x + ch * plane;
  const float* yc = y + ch * plane;
  const int ox = blockIdx.x * kT - kR, oy = blockIdx.y * kT - kR;
  {
    // every halo load is issued before the first LDS store (clamped addresses,
    // zero outside the image), so their latencies overlap
    float vx[kLoads], vy[kLoads];
#pragma unroll
    for (int q = 0; q < kLoads; ++q) {
      const size_t o = halo_offset(threadIdx.x + q * 256, ox, oy, W, H);
      vx[q] = xc[o];
      vy[q] = yc[o];
    }
#pragma unroll
    for (int q = 0; q < kLoads; ++q) {
      const int t = threadIdx.x + q * 256;
      if (t < kH * kH) {
        const bool in = halo_inside(t, ox, oy, W, H);
        sx[t / kH][t % kH] = in ? vx[q] : 0.f;
        sy[t / kH][t % kH] = in ? vy[q] : 0.f;
      }
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < kH * kT; t += 256) {
    const int r = t / kT, c = t % kT;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, a4 = 0.f;
#pragma unroll
    for (int i = 0; i < kN; ++i) {
      const float xv = sx[r][c + i], yv = sy[r][c + i];
      const float wx = win.w[i] * xv, wy = win.w[i] * yv;
      a0 += wx;
      a1 += wy;
      a2 = fmaf(wx, xv, a2);
      a3 = fmaf(wy, yv, a3);
      a4 = fmaf(wx, yv, a4);
    }
    hq[0][r][c] = a0;
    hq[1][r][c] = a1;
    hq[2][r][c] = a2;
    hq[3][r][c] = a3;
    hq[4][r][c] = a4;
  }
  __syncthreads();
  int c, r0;
  vert_slot(c, r0);
  float mom[kRows][5];
  vert_filter<5>(hq, win, c, r0, mom);
  double l1 = 0.0, ss = 0.0;
  const int gx = blockIdx.x * kT + c;
#pragma unroll
  for (int o = 0; o < kRows; ++o) {
    const int gy = blockIdx.y * kT + r0 + o;
    if (gx < W && gy < H) {
      const float mx = mom[o][0], my = mom[o][1];
      const float sxx = mom[o][2] - mx * mx, syy = mom[o][3] - my * my;
      const float sxy = mom[o][4] - mx * my;
      const float A1 = 2.f * mx * my + kC1, A2 = 2.f * sxy + kC2;
      const float B1 = mx * mx + my * my + kC1, B2 = sxx + syy + kC2;
      // With P = 1/(B1 B2) and S = A1 A2 P:
      //   dS/dmu_x = 2 P my (A2 - A1) + 2 S mx (1/B2 - 1/B1),
      //   dS/dE[x^2] = -S / B2,  dS/dE[xy] = 2 A1 P,
      // so only B1 >= C1 and B2 >= C2 are inverted (A2 = 2 sigma_xy + C2 may vanish).
      const float iB1 = __builtin_amdgcn_rcpf(B1), iB2 = __builtin_amdgcn_rcpf(B2);
      const float Pb = iB1 * iB2;
      const float S = (A1 * A2) * Pb;
      const float g1 = 2.f * (my * (A2 - A1) * Pb + S * mx * (iB2 - iB1));
      const float g2 = -S * iB2;
      const float g3 = 2.f * A1 * Pb;
      const size_t pix = (size_t)gy * W + gx;
      gmap[(0 * 3 + ch) * plane + pix] = g1;
      gmap[(1 * 3 + ch) * plane + pix] = g2;
      gmap[(2 * 3 + ch) * plane + pix] = g3;
      l1 += fabs((double)sx[r0 + o + kR][c + kR] - (double)sy[r0 + o + kR][c + kR]);
      ss += (double)S;
    }
  }
  // block reduction of the two sums
  __shared__ double red[2][4];
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    l1 += __shfl_xor(l1, d, 64);
    ss += __shfl_xor(ss, d, 64);
  }
  const int lane = __lane_id(), wave = threadIdx.x / 64;
  if (lane == 0) {
    red[0][wave] = l1;
    red[1][wave] = ss;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const size_t b = ((size_t)ch * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    part[2 * b + 0] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    part[2 * b + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  }
}

__global__ __launch_bounds__(256) void k_ssim_bwd(const float* __restrict__ x,
                                                  const float* __restrict__ y, int W, int H,
                                                  Win win, const float* __restrict__ gmap,
                                                  float lambda, float scale,
                                                  float* __restrict__ dl) {
  __shared__ float sg[3][kH][kP];
  __shared__ float hq[3][kH][kQ];
  const int ch = blockIdx.z;
  const size_t plane = (size_t)W * H;
  const int ox = blockIdx.x * kT - kR, oy = blockIdx.y * kT - kR;
  {
    float v[3][kLoads];
#pragma unroll
    for (int q = 0; q < kLoads; ++q) {
      const size_t o = halo_offset(threadIdx.x + q * 256, ox, oy, W, H);
#pragma unroll
      for (int m = 0; m < 3; ++m) v[m][q] = gmap[(m * 3 + ch) * plane + o];
    }
#pragma unroll
    for (int q = 0; q < kLoads; ++q) {
      const int t = threadIdx.x + q * 256;
      if (t < kH * kH) {
        const bool in = halo_inside(t, ox, oy, W, H);
#pragma unroll
        for (int m = 0; m < 3; ++m) sg[m][t / kH][t % kH] = in ? v[m][q] : 0.f;
      }
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < kH * kT; t += 256) {
    const int r = t / kT, c = t % kT;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
    for (int i = 0; i < kN; ++i) {
      const float w = win.w[i];
      a0 = fmaf(w, sg[0][r][c + i], a0);
      a1 = fmaf(w, sg[1][r][c + i], a1);
      a2 = fmaf(w, sg[2][r][c + i], a2);
    }
    hq[0][r][c] = a0;
    hq[1][r][c] = a1;
    hq[2][r][c] = a2;
  }
  __syncthreads();
  int c, r0;
  vert_slot(c, r0);
  float f[kRows][3];
  vert_filter<3>(hq, win, c, r0, f);
  const int gx = blockIdx.x * kT + c;
  if (gx >= W) return;
#pragma unroll
  for (int o = 0; o < kRows; ++o) {
    const int gy = blockIdx.y * kT + r0 + o;
    if (gy >= H) break;
    const size_t pix = ch * plane + (size_t)gy * W + gx;
    const float xv = x[pix], yv = y[pix];
    const float sgn = (xv > yv) ? 1.f : ((xv < yv) ? -1.f : 0.f);
    dl[pix] = scale * ((1.f - lambda) * sgn - lambda * (f[o][0] + 2.f * xv * f[o][1] + yv * f[o][2]));
  }
}

struct LossRed {
  int nv;
  int nblk[kMaxViews];
  long long off[kMaxViews];
  double inv_count[kMaxViews];
};

constexpr int kRedBlocks = 64;

__device__ inline void block_sum2(double& a, double& b) {
  __shared__ double sh[2][256];
  sh[0][threadIdx.x] = a;
  sh[1][threadIdx.x] = b;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + st];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + st];
    }
    __syncthreads();
  }
  a = sh[0][0];
  b = sh[1][0];
  __syncthreads();
}

// Stage 1: block (b, v) sums view v's partials b, b + 64, ... (fixed order).
__global__ __launch_bounds__(256) void k_loss_partial(const double* __restrict__ part, LossRed lr,
                                                      double* __restrict__ part2) {
  const int v = blockIdx.y;
  double a = 0.0, b = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < lr.nblk[v]; i += kRedBlocks * 256) {
    a += part[2 * (lr.off[v] + i) + 0];
    b += part[2 * (lr.off[v] + i) + 1];
  }
  block_sum2(a, b);
  if (threadIdx.x == 0) {
    part2[2 * (v * kRedBlocks + blockIdx.x) + 0] = a;
    part2[2 * (v * kRedBlocks + blockIdx.x) + 1] = b;
  }
}

// Stage 2: one block combines the per-view sums into the loss.
__global__ __launch_bounds__(256) void k_loss_final(const double* __restrict__ part2, LossRed lr,
                                                    float lambda, float* __restrict__ out) {
  double total = 0.0;
  for (int v = 0; v < lr.nv; ++v) {
    double a = 0.0, b = 0.0;
    if (threadIdx.x < kRedBlocks) {
      a = part2[2 * (v * kRedBlocks + threadIdx.x) + 0];
      b = part2[2 * (v * kRedBlocks + threadIdx.x) + 1];
    }
    block_sum2(a, b);
    total += (1.0 - lambda) * a * lr.inv_count[v] + lambda * (1.0 - b * lr.inv_count[v]);
  }
  if (threadIdx.x == 0) *out = (float)(total / lr.nv);
}

}  // namespace

struct LossScratch {
  DevBuf gmap, part;
};

// One scratch per context, kept for the context's lifetime.
static LossScratch& loss_scratch(Ctx* ctx) {
  return *reinterpret_cast<LossScratch*>(ctx->loss_scratch);
}

gs_status launch_loss(Ctx* ctx, const float* const* x, const float* const* y, const int* W,
                      const int* H, int nv, float lambda, float* loss_out, float* const* dl,
                      hipStream_t s) {
  Win win;
  {
    double g[kN], sum = 0.0;
    for (int i = 0; i < kN; ++i) {
      const double d = i - kR;
      g[i] = exp(-(d * d) / (2.0 * 1.5 * 1.5));
      sum += g[i];
    }
    for (int i = 0; i < kN; ++i) win.w[i] = (float)(g[i] / sum);
  }
  if (ctx->loss_scratch == nullptr) ctx->loss_scratch = new LossScratch();
  LossScratch& ls = loss_scratch(ctx);
  size_t max_plane = 0, total_blocks = 0;
  LossRed lr;
  lr.nv = nv;
  for (int v = 0; v < nv; ++v) {
    const size_t plane = (size_t)W[v] * H[v];
    if (plane > max_plane) max_plane = plane;
    const int nbx = (W[v] + kT - 1) / kT, nby = (H[v] + kT - 1) / kT;
    lr.nblk[v] = nbx * nby * 3;
    lr.off[v] = (long long)total_blocks;
    lr.inv_count[v] = 1.0 / (3.0 * (double)plane);
    total_blocks += (size_t)lr.nblk[v];
  }
  gs_status st = buf_ensure(ctx, ls.gmap, sizeof(float) * 9 * max_plane);
  if (st != GS_OK) return st;
  st = buf_ensure(ctx, ls.part, sizeof(double) * 2 * (total_blocks + kRedBlocks * kMaxViews));
  if (st != GS_OK) return st;
  double* part2 = (double*)ls.part.p + 2 * total_blocks;
  for (int v = 0; v < nv; ++v) {
    const dim3 grid((W[v] + kT - 1) / kT, (H[v] + kT - 1) / kT, 3);
    hipLaunchKernelGGL(k_ssim_fwd, grid, dim3(256), 0, s, x[v], y[v], W[v], H[v], win,
                       (float*)ls.gmap.p, (double*)ls.part.p + 2 * lr.off[v]);
    GS_LAUNCHED("ssim_fwd");
    if (dl != nullptr && dl[v] != nullptr) {
      const float scale = (float)(1.0 / (3.0 * (double)W[v] * H[v] * nv));
      hipLaunchKernelGGL(k_ssim_bwd, grid, dim3(256), 0, s, x[v], y[v], W[v], H[v], win,
                         (const float*)ls.gmap.p, lambda, scale, dl[v]);
      GS_LAUNCHED("ssim_bwd");
    }
  }
  if (loss_out != nullptr) {
    hipLaunchKernelGGL(k_loss_partial, dim3(kRedBlocks, nv), dim3(256), 0, s,
                       (const double*)ls.part.p, lr, part2);
    GS_LAUNCHED("loss_partial");
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, s, (const double*)part2, lr, lambda,
                       loss_out);
    GS_LAUNCHED("loss_final");
  }
  return GS_OK;
}

void free_loss_scratch(Ctx* ctx) {
  if (ctx->loss_scratch == nullptr) return;
  LossScratch* ls = reinterpret_cast<LossScratch*>(ctx->loss_scratch);
  buf_free(ctx, ls->gmap);
  buf_free(ctx, ls->part);
  delete ls;
  ctx->loss_scratch = nullptr;
}

}  // namespace isogs
