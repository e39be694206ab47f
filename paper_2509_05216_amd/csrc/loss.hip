// Training loss: mean over views of (1 - lambda) L1 + lambda (1 - SSIM), and its
// gradient with respect to the rendered image.
//
// SSIM uses an 11 x 11 Gaussian window (sigma 1.5, separable, weights summing
// to one), C1 = 0.01^2, C2 = 0.03^2, zero padding, averaged over pixels and
// channels.  Two LDS-tiled passes per view (16 x 16 output pixels per block,
// a 26 x 26 halo tile): the first forms the five local moments by separable
// filtering and writes, per pixel, the partials g1 = dS/dmu_x, g2 = dS/dE[x^2]
// and g3 = dS/dE[xy]; the second filters those maps (the window is symmetric,
// so the zero-padded correlation is its own adjoint) and combines them with
// the L1 term:  dL/dx = s [(1 - lambda) sign(x - y)
//                          - lambda (w*g1 + 2 x w*g2 + y w*g3)],  s = 1/(3 H W V).
// Loss sums are reduced per block into float64 partials and summed by a final
// single-block kernel, so the loss value is deterministic.
#include "internal.h"

namespace isogs {
namespace {

constexpr int kB = 16;           // output tile side
constexpr int kR = 5;            // window radius
constexpr int kS = kB + 2 * kR;  // 26: halo tile side
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;

struct Win {
  float w[2 * kR + 1];
};

__global__ __launch_bounds__(256) void k_ssim_fwd(const float* __restrict__ x,
                                                  const float* __restrict__ y, int W, int H,
                                                  Win win, float* __restrict__ gmap,
                                                  double* __restrict__ part) {
  __shared__ float sx[kS][kS], sy[kS][kS];
  __shared__ float hq[5][kS][kB];
  const int ch = blockIdx.z;
  const size_t plane = (size_t)W * H;
  const float* xc = x + ch * plane;
  const float* yc = y + ch * plane;
  const int ox = blockIdx.x * kB - kR, oy = blockIdx.y * kB - kR;
  for (int t = threadIdx.x; t < kS * kS; t += 256) {
    const int r = t / kS, c = t % kS;
    const int gx = ox + c, gy = oy + r;
    const bool in = gx >= 0 && gx < W && gy >= 0 && gy < H;
    sx[r][c] = in ? xc[(size_t)gy * W + gx] : 0.f;
    sy[r][c] = in ? yc[(size_t)gy * W + gx] : 0.f;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < kS * kB; t += 256) {
    const int r = t / kB, c = t % kB;
    float a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0;
#pragma unroll
    for (int i = 0; i < 2 * kR + 1; ++i) {
      const float xv = sx[r][c + i], yv = sy[r][c + i], w = win.w[i];
      a0 += w * xv;
      a1 += w * yv;
      a2 += w * xv * xv;
      a3 += w * yv * yv;
      a4 += w * xv * yv;
    }
    hq[0][r][c] = a0; hq[1][r][c] = a1; hq[2][r][c] = a2; hq[3][r][c] = a3; hq[4][r][c] = a4;
  }
  __syncthreads();
  const int r = threadIdx.x / kB, c = threadIdx.x % kB;
  const int gx = blockIdx.x * kB + c, gy = blockIdx.y * kB + r;
  float mx = 0, my = 0, exx = 0, eyy = 0, exy = 0;
#pragma unroll
  for (int i = 0; i < 2 * kR + 1; ++i) {
    const float w = win.w[i];
    mx += w * hq[0][r + i][c];
    my += w * hq[1][r + i][c];
    exx += w * hq[2][r + i][c];
    eyy += w * hq[3][r + i][c];
    exy += w * hq[4][r + i][c];
  }
  double l1 = 0.0, ss = 0.0;
  if (gx < W && gy < H) {
    const float sxx = exx - mx * mx, syy = eyy - my * my, sxy = exy - mx * my;
    const float A1 = 2.f * mx * my + kC1, A2 = 2.f * sxy + kC2;
    const float B1 = mx * mx + my * my + kC1, B2 = sxx + syy + kC2;
    const float S = (A1 * A2) / (B1 * B2);
    const float g1 = S * (2.f * my / A1 - 2.f * my / A2 - 2.f * mx / B1 + 2.f * mx / B2);
    const float g2 = -S / B2;
    const float g3 = 2.f * S / A2;
    const size_t pix = (size_t)gy * W + gx;
    gmap[(0 * 3 + ch) * plane + pix] = g1;
    gmap[(1 * 3 + ch) * plane + pix] = g2;
    gmap[(2 * 3 + ch) * plane + pix] = g3;
    l1 = fabs((double)sx[r + kR][c + kR] - (double)sy[r + kR][c + kR]);
    ss = (double)S;
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
  __shared__ float sg[3][kS][kS];
  __shared__ float hq[3][kS][kB];
  const int ch = blockIdx.z;
  const size_t plane = (size_t)W * H;
  const int ox = blockIdx.x * kB - kR, oy = blockIdx.y * kB - kR;
  for (int t = threadIdx.x; t < kS * kS; t += 256) {
    const int r = t / kS, c = t % kS;
    const int gx = ox + c, gy = oy + r;
    const bool in = gx >= 0 && gx < W && gy >= 0 && gy < H;
    const size_t pix = (size_t)gy * W + gx;
#pragma unroll
    for (int m = 0; m < 3; ++m) sg[m][r][c] = in ? gmap[(m * 3 + ch) * plane + pix] : 0.f;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < kS * kB; t += 256) {
    const int r = t / kB, c = t % kB;
    float a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
    for (int i = 0; i < 2 * kR + 1; ++i) {
      const float w = win.w[i];
      a0 += w * sg[0][r][c + i];
      a1 += w * sg[1][r][c + i];
      a2 += w * sg[2][r][c + i];
    }
    hq[0][r][c] = a0; hq[1][r][c] = a1; hq[2][r][c] = a2;
  }
  __syncthreads();
  const int r = threadIdx.x / kB, c = threadIdx.x % kB;
  const int gx = blockIdx.x * kB + c, gy = blockIdx.y * kB + r;
  if (gx >= W || gy >= H) return;
  float f1 = 0, f2 = 0, f3 = 0;
#pragma unroll
  for (int i = 0; i < 2 * kR + 1; ++i) {
    const float w = win.w[i];
    f1 += w * hq[0][r + i][c];
    f2 += w * hq[1][r + i][c];
    f3 += w * hq[2][r + i][c];
  }
  const size_t pix = ch * plane + (size_t)gy * W + gx;
  const float xv = x[pix], yv = y[pix];
  const float sgn = (xv > yv) ? 1.f : ((xv < yv) ? -1.f : 0.f);
  dl[pix] = scale * ((1.f - lambda) * sgn - lambda * (f1 + 2.f * xv * f2 + yv * f3));
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
    double g[2 * kR + 1], sum = 0.0;
    for (int i = 0; i < 2 * kR + 1; ++i) {
      const double d = i - kR;
      g[i] = exp(-(d * d) / (2.0 * 1.5 * 1.5));
      sum += g[i];
    }
    for (int i = 0; i < 2 * kR + 1; ++i) win.w[i] = (float)(g[i] / sum);
  }
  if (ctx->loss_scratch == nullptr) ctx->loss_scratch = new LossScratch();
  LossScratch& ls = loss_scratch(ctx);
  size_t max_plane = 0, total_blocks = 0;
  LossRed lr;
  lr.nv = nv;
  for (int v = 0; v < nv; ++v) {
    const size_t plane = (size_t)W[v] * H[v];
    if (plane > max_plane) max_plane = plane;
    const int nbx = (W[v] + kB - 1) / kB, nby = (H[v] + kB - 1) / kB;
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
    const dim3 grid((W[v] + kB - 1) / kB, (H[v] + kB - 1) / kB, 3);
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
