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
// A horizontal task makes four outputs of one halo row from 14 inputs (read
// 8 bytes at a time, with x^2, y^2 and x y formed once per input), each tap an
// explicit fused multiply-add per moment.  In the vertical pass each thread
// produces four consecutive rows of one column from 14 LDS rows.  Loss sums are reduced per block into
// float64 partials and summed by a final single-block kernel, so the loss
// value is deterministic.
#include <atomic>

#include "internal.h"

namespace isogs {
namespace {

constexpr int kT = 32;           // output tile side
constexpr int kR = 5;            // window radius
constexpr int kN = 2 * kR + 1;   // taps
constexpr int kH = kT + 2 * kR;  // 42: halo tile side (LDS rows of 168 bytes, 8-byte aligned)
constexpr int kQ = kT + 4;       // 36: LDS row of the horizontal pass (16-byte aligned)
constexpr int kRows = 4;         // output rows per thread in the vertical pass
constexpr int kGroups = kT / 4;  // four-wide output groups per row in the horizontal pass
constexpr int kHTasks = kH * kGroups;  // 336 horizontal tasks (halo row, group)
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;

struct Win {
  float w[kN];
};

// Halo tiles are loaded by rows: wave w takes rows w, w + 4, ..., lane l
// column l (lanes 42-63 load a valid clamped address and store nothing), so
// the column clamp is a per-lane constant and the row clamp a scalar.
constexpr int kHaloRows = (kH + 3) / 4;  // 11 rows per wave

struct HaloCols {
  uint32_t gxc;  // clamped image column of this lane
  bool inx;      // lane < 42 and its column inside the image
};

__device__ inline HaloCols halo_cols(int ox, int W) {
  const int lane = (int)(threadIdx.x % 64);
  const int gx = ox + lane;
  return {(uint32_t)min(max(gx, 0), W - 1), lane < kH && gx >= 0 && gx < W};
}

// This thread's share of a halo tile of NI image planes (top-left halo pixel
// row oy), into registers; the loads are issued together.
template <int NI>
__device__ inline void halo_load(const float* const (&img)[NI], HaloCols hc, int oy, int W, int H,
                                 float (&v)[NI][kHaloRows]) {
  // wave-uniform (scalar) row arithmetic; per lane only the column offset
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
#pragma unroll
  for (int k = 0; k < kHaloRows; ++k) {
    const int gy = min(max(oy + wave + 4 * k, 0), H - 1);
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const float* rp = img[i] + (size_t)gy * W;
      v[i][k] = rp[hc.gxc];
    }
  }
  // keep every load here, ahead of the (predicated) stores, so that their
  // latencies overlap instead of each store waiting for its own load
#pragma unroll
  for (int k = 0; k < kHaloRows; ++k)
#pragma unroll
    for (int i = 0; i < NI; ++i) asm volatile("" : "+v"(v[i][k]));
}

// ... and from registers into LDS tiles, zero outside the image.
template <int NI>
__device__ inline void halo_store(float (*const (&tile)[NI])[kH], const float (&v)[NI][kHaloRows],
                                  HaloCols hc, int oy, int H) {
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
  const int lane = (int)(threadIdx.x % 64);
#pragma unroll
  for (int k = 0; k < kHaloRows; ++k) {
    const int r = wave + 4 * k;
    const bool in = hc.inx && oy + r >= 0 && oy + r < H;
    if (lane < kH && r < kH) {
#pragma unroll
      for (int i = 0; i < NI; ++i) tile[i][r][lane] = in ? v[i][k] : 0.f;
    }
  }
}

// Columns c0 .. c0 + 13 of row r of an LDS halo tile (c0 a multiple of 4, so
// the seven 8-byte reads are aligned): the inputs of four horizontal outputs.
__device__ inline void row14(const float (*tile)[kH], int r, int c0, float (&v)[14]) {
  const float2* p = reinterpret_cast<const float2*>(&tile[r][c0]);
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    const float2 u = p[k];
    v[2 * k] = u.x;
    v[2 * k + 1] = u.y;
  }
}

// Tile (bx, by) and channel bz of this block.  Workgroups are dispatched to
// the eight XCDs (each with its own L2) in turn, so consecutive block indices
// go to different XCDs; the permutation below gives each XCD a contiguous run
// of tiles instead, so that the halos neighbouring tiles share are read into
// the same L2.  A bijection (the last total % 8 blocks keep their place), so
// every tile is done once whatever the dispatch order.
__device__ inline void xcd_tile(int& bx, int& by, int& bz) {
  const uint32_t gx = gridDim.x, gxy = gridDim.x * gridDim.y;
  const uint32_t total = gxy * gridDim.z;
  const uint32_t L = blockIdx.x + gx * (blockIdx.y + gridDim.y * blockIdx.z);
  const uint32_t n8 = total / 8;
  const uint32_t T = L < 8 * n8 ? (L % 8) * n8 + L / 8 : L;
  bz = (int)(T / gxy);
  const uint32_t r = T % gxy;
  by = (int)(r / gx);
  bx = (int)(r % gx);
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

// One block per 32 x 32 tile and channel.
__global__ __launch_bounds__(256) void k_ssim_fwd(const float* __restrict__ x,
                                                  const float* __restrict__ y, int W, int H,
                                                  Win win, float* __restrict__ gmap,
                                                  double* __restrict__ part) {
  __shared__ alignas(16) float sx[kH][kH];
  __shared__ alignas(16) float sy[kH][kH];
  __shared__ alignas(16) float hq[5][kH][kQ];
  int bx, by, ch;
  xcd_tile(bx, by, ch);
  const size_t plane = (size_t)W * H;
  const int ox = bx * kT - kR, oy = by * kT - kR;
  {
    // every halo load is issued before the first LDS store (clamped addresses,
    // zero outside the image), so their latencies overlap
    const HaloCols hc = halo_cols(ox, W);
    const float* const src[2] = {x + ch * plane, y + ch * plane};
    float (*const dst[2])[kH] = {sx, sy};
    float v[2][kHaloRows];
    halo_load<2>(src, hc, oy, W, H, v);
    halo_store<2>(dst, v, hc, oy, H);
  }
  __syncthreads();
  // horizontal pass: four outputs of one halo row per task; the products x^2,
  // y^2, x y are formed once per input, so each tap is five fused multiply-adds
  for (int t = threadIdx.x; t < kHTasks; t += 256) {
    const int r = t / kGroups, c0 = (t % kGroups) * 4;
    float xv[14], yv[14];
    row14(sx, r, c0, xv);
    row14(sy, r, c0, yv);
    float xx[14], yy[14], xy[14];
#pragma unroll
    for (int k = 0; k < 14; ++k) {
      xx[k] = xv[k] * xv[k];
      yy[k] = yv[k] * yv[k];
      xy[k] = xv[k] * yv[k];
    }
    float a0[4], a1[4], a2[4], a3[4], a4[4];
#pragma unroll
    for (int o = 0; o < 4; ++o) a0[o] = a1[o] = a2[o] = a3[o] = a4[o] = 0.f;
#pragma unroll
    for (int i = 0; i < kN; ++i)
#pragma unroll
      for (int o = 0; o < 4; ++o) {
        const float w = win.w[i];
        a0[o] = fmaf(w, xv[o + i], a0[o]);
        a1[o] = fmaf(w, yv[o + i], a1[o]);
        a2[o] = fmaf(w, xx[o + i], a2[o]);
        a3[o] = fmaf(w, yy[o + i], a3[o]);
        a4[o] = fmaf(w, xy[o + i], a4[o]);
      }
    *reinterpret_cast<float4*>(&hq[0][r][c0]) = make_float4(a0[0], a0[1], a0[2], a0[3]);
    *reinterpret_cast<float4*>(&hq[1][r][c0]) = make_float4(a1[0], a1[1], a1[2], a1[3]);
    *reinterpret_cast<float4*>(&hq[2][r][c0]) = make_float4(a2[0], a2[1], a2[2], a2[3]);
    *reinterpret_cast<float4*>(&hq[3][r][c0]) = make_float4(a3[0], a3[1], a3[2], a3[3]);
    *reinterpret_cast<float4*>(&hq[4][r][c0]) = make_float4(a4[0], a4[1], a4[2], a4[3]);
  }
  __syncthreads();
  int c, r0;
  vert_slot(c, r0);
  float mom[kRows][5];
  vert_filter<5>(hq, win, c, r0, mom);
  double l1 = 0.0, ss = 0.0;
  const int gx = bx * kT + c;
#pragma unroll
  for (int o = 0; o < kRows; ++o) {
    const int gy = by * kT + r0 + o;
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
    const size_t b = ((size_t)ch * gridDim.y + by) * gridDim.x + bx;
    part[2 * b + 0] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    part[2 * b + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  }
}

__global__ __launch_bounds__(256) void k_ssim_bwd(const float* __restrict__ x,
                                                  const float* __restrict__ y, int W, int H,
                                                  Win win, const float* __restrict__ gmap,
                                                  float lambda, float scale,
                                                  float* __restrict__ dl) {
  __shared__ alignas(16) float sg[3][kH][kH];
  __shared__ alignas(16) float hq[3][kH][kQ];
  int bx, by, ch;
  xcd_tile(bx, by, ch);
  const size_t plane = (size_t)W * H;
  const int ox = bx * kT - kR, oy = by * kT - kR;
  {
    const HaloCols hc = halo_cols(ox, W);
    const float* const src[3] = {gmap + (size_t)(0 * 3 + ch) * plane,
                                 gmap + (size_t)(1 * 3 + ch) * plane,
                                 gmap + (size_t)(2 * 3 + ch) * plane};
    float (*const dst[3])[kH] = {sg[0], sg[1], sg[2]};
    float v[3][kHaloRows];
    halo_load<3>(src, hc, oy, W, H, v);
    halo_store<3>(dst, v, hc, oy, H);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < kHTasks; t += 256) {
    const int r = t / kGroups, c0 = (t % kGroups) * 4;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      float gv[14];
      row14(sg[m], r, c0, gv);
      float a[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int i = 0; i < kN; ++i)
#pragma unroll
        for (int o = 0; o < 4; ++o) a[o] = fmaf(win.w[i], gv[o + i], a[o]);
      *reinterpret_cast<float4*>(&hq[m][r][c0]) = make_float4(a[0], a[1], a[2], a[3]);
    }
  }
  __syncthreads();
  int c, r0;
  vert_slot(c, r0);
  float f[kRows][3];
  vert_filter<3>(hq, win, c, r0, f);
  const int gx = bx * kT + c;
  if (gx >= W) return;
#pragma unroll
  for (int o = 0; o < kRows; ++o) {
    const int gy = by * kT + r0 + o;
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

// Image-quality metrics: block (b, v) sums (x - y)^2 over view v's values
// b * 256 + t, b * 256 + t + 64 * 256, ... (fixed order) in float64.
struct ImagePtrs {
  const float* x[kMaxViews];
  const float* y[kMaxViews];
};

__global__ __launch_bounds__(256) void k_sq_partial(ImagePtrs im, LossRed lr,
                                                    double* __restrict__ part3) {
  const int v = blockIdx.y;
  const float* x = im.x[v];
  const float* y = im.y[v];
  const long long count = (long long)(0.5 + 1.0 / lr.inv_count[v]);
  double a = 0.0, b = 0.0;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < count;
       i += (long long)kRedBlocks * 256) {
    const double d = (double)x[i] - (double)y[i];
    a += d * d;
  }
  block_sum2(a, b);
  if (threadIdx.x == 0) part3[v * kRedBlocks + blockIdx.x] = a;
}

// Block v: mse, psnr = 10 log10(1 / mse), mean |x - y| and mean SSIM of view v.
__global__ __launch_bounds__(256) void k_metrics_final(const double* __restrict__ part2,
                                                       const double* __restrict__ part3,
                                                       LossRed lr, float* __restrict__ out) {
  const int v = blockIdx.x;
  double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
  if (threadIdx.x < kRedBlocks) {
    a = part2[2 * (v * kRedBlocks + threadIdx.x) + 0];
    b = part2[2 * (v * kRedBlocks + threadIdx.x) + 1];
    c = part3[v * kRedBlocks + threadIdx.x];
  }
  block_sum2(a, b);
  block_sum2(c, d);
  if (threadIdx.x == 0) {
    const double mse = c * lr.inv_count[v];
    out[4 * v + 0] = (float)mse;
    out[4 * v + 1] = (float)(mse > 0.0 ? -10.0 * log10(mse) : INFINITY);
    out[4 * v + 2] = (float)(a * lr.inv_count[v]);
    out[4 * v + 3] = (float)(b * lr.inv_count[v]);
  }
}

}  // namespace

void loss_scratch_bytes(const int* W, const int* H, int nv, size_t* gmap_bytes,
                        size_t* part_bytes) {
  size_t max_plane = 0, total_blocks = 0;
  for (int v = 0; v < nv; ++v) {
    const size_t plane = (size_t)W[v] * H[v];
    if (plane > max_plane) max_plane = plane;
    total_blocks += (size_t)((W[v] + kT - 1) / kT) * ((H[v] + kT - 1) / kT) * 3;
  }
  *gmap_bytes = sizeof(float) * 9 * max_plane;
  // block partials (2 each), per-view stage-1 sums (2 each), metric sums (1 each)
  *part_bytes = sizeof(double) * (2 * (total_blocks + kRedBlocks * kMaxViews) +
                                  (size_t)kRedBlocks * kMaxViews);
}

gs_status loss_reserve(Ctx* ctx, LossScratch& ls, const int* W, const int* H, int nv,
                       hipStream_t s) {
  if (ls.last_use == nullptr)
    GS_HIP(hipEventCreateWithFlags(&ls.last_use, hipEventDisableTiming));
  size_t gb = 0, pb = 0;
  loss_scratch_bytes(W, H, nv, &gb, &pb);
  gs_status st = buf_ensure(ctx, ls.gmap, gb, s, ls.last_use);
  if (st != GS_OK) return st;
  return buf_ensure(ctx, ls.part, pb, s, ls.last_use);
}

gs_status launch_loss(const LossScratch& ls, const float* const* x, const float* const* y,
                      const int* W, const int* H, int nv, float lambda, float* loss_out,
                      float* const* dl, hipStream_t s) {
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
  size_t total_blocks = 0;
  LossRed lr;
  lr.nv = nv;
  for (int v = 0; v < nv; ++v) {
    const size_t plane = (size_t)W[v] * H[v];
    const int nbx = (W[v] + kT - 1) / kT, nby = (H[v] + kT - 1) / kT;
    lr.nblk[v] = nbx * nby * 3;
    lr.off[v] = (long long)total_blocks;
    lr.inv_count[v] = 1.0 / (3.0 * (double)plane);
    total_blocks += (size_t)lr.nblk[v];
  }
  {
    size_t gb = 0, pb = 0;
    loss_scratch_bytes(W, H, nv, &gb, &pb);
    if (ls.gmap.cap < gb || ls.part.cap < pb) {
      set_error("internal: loss workspace of %zu / %zu bytes is smaller than %zu / %zu",
                ls.gmap.cap, ls.part.cap, gb, pb);
      return GS_ERR_CAPACITY;
    }
  }
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

// ---------------------------------------------------------- fixed workspace
// Workspace of gs_loss_grad_noalloc: one file-scope device array per GPU, held
// for the life of the process, so that call allocates nothing.  In host code
// `scratch` names a host-side stand-in, never the device array: its device
// address comes from hipGetSymbolAddress, taken once per device with that
// device current (loss_noalloc_setup, called when a context is created) and
// kept in g_noalloc_ptr.
constexpr size_t kNoAllocGmapBytes = sizeof(float) * 9 * kNoAllocMaxPixels;
// 2048 output tiles cover any view of <= 2^20 pixels whose sides are <= 16384
// (ceil(W/32) ceil(H/32) <= 1536 there)
constexpr size_t kNoAllocPartBytes =
    sizeof(double) * (2 * ((size_t)kMaxViews * 3 * 2048 + (size_t)kRedBlocks * kMaxViews) +
                      (size_t)kRedBlocks * kMaxViews);
constexpr size_t kNoAllocBytes = kNoAllocGmapBytes + kNoAllocPartBytes;
static_assert(kNoAllocGmapBytes % 256 == 0, "partials start 256-byte aligned");

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kNoAllocDevices = 64;
static std::atomic<void*> g_noalloc_ptr[kNoAllocDevices];

gs_status loss_noalloc_setup(int device) {
  if (device < 0 || device >= kNoAllocDevices) {
    set_error("device %d: the fixed loss workspace supports devices 0..%d", device,
              kNoAllocDevices - 1);
    return GS_ERR_UNSUPPORTED;
  }
  if (g_noalloc_ptr[device].load(std::memory_order_acquire) != nullptr) return GS_OK;
  static std::mutex mu;
  std::lock_guard<std::mutex> lk(mu);
  if (g_noalloc_ptr[device].load(std::memory_order_relaxed) != nullptr) return GS_OK;
  int cur = -1;
  GS_HIP(hipGetDevice(&cur));
  if (cur != device) {
    set_error("internal: loss_noalloc_setup(%d) with device %d current", device, cur);
    return GS_ERR_INVALID;
  }
  void* ptr = nullptr;
  GS_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (ptr == nullptr) {
    set_error("hipGetSymbolAddress returned no address for the loss workspace");
    return GS_ERR_HIP;
  }
  g_noalloc_ptr[device].store(ptr, std::memory_order_release);
  return GS_OK;
}

gs_status loss_noalloc_workspace(int device, const int* W, const int* H, int nv,
                                 LossScratch* out) {
  size_t gb = 0, pb = 0;
  loss_scratch_bytes(W, H, nv, &gb, &pb);
  if (gb > kNoAllocGmapBytes || pb > kNoAllocPartBytes) {
    set_error("gs_loss_grad_noalloc: views need a %zu + %zu byte workspace; the fixed one "
              "holds %zu + %zu bytes (at most %zu pixels per view)", gb, pb,
              kNoAllocGmapBytes, kNoAllocPartBytes, kNoAllocMaxPixels);
    return GS_ERR_CAPACITY;
  }
  void* base = (device >= 0 && device < kNoAllocDevices)
                   ? g_noalloc_ptr[device].load(std::memory_order_acquire)
                   : nullptr;
  if (base == nullptr) {
    set_error("gs_loss_grad_noalloc: the fixed workspace of device %d was not set up", device);
    return GS_ERR_INVALID;
  }
  out->gmap.p = base;
  out->gmap.cap = kNoAllocGmapBytes;
  out->part.p = (unsigned char*)base + kNoAllocGmapBytes;
  out->part.cap = kNoAllocPartBytes;
  out->last_use = nullptr;
  return GS_OK;
}

gs_status launch_metrics(const LossScratch& ls, const float* const* x, const float* const* y,
                         const int* W, const int* H, int nv, float* out, hipStream_t s) {
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
  size_t total_blocks = 0;
  LossRed lr;
  lr.nv = nv;
  for (int v = 0; v < nv; ++v) {
    const size_t plane = (size_t)W[v] * H[v];
    lr.nblk[v] = ((W[v] + kT - 1) / kT) * ((H[v] + kT - 1) / kT) * 3;
    lr.off[v] = (long long)total_blocks;
    lr.inv_count[v] = 1.0 / (3.0 * (double)plane);
    total_blocks += (size_t)lr.nblk[v];
  }
  size_t gb = 0, pb = 0;
  loss_scratch_bytes(W, H, nv, &gb, &pb);
  if (ls.gmap.cap < gb || ls.part.cap < pb) {
    set_error("internal: metrics workspace too small");
    return GS_ERR_CAPACITY;
  }
  double* part = (double*)ls.part.p;
  double* part2 = part + 2 * total_blocks;
  double* part3 = part2 + 2 * (size_t)kRedBlocks * kMaxViews;
  for (int v = 0; v < nv; ++v) {
    const dim3 grid((W[v] + kT - 1) / kT, (H[v] + kT - 1) / kT, 3);
    hipLaunchKernelGGL(k_ssim_fwd, grid, dim3(256), 0, s, x[v], y[v], W[v], H[v], win,
                       (float*)ls.gmap.p, part + 2 * lr.off[v]);
    GS_LAUNCHED("ssim_fwd");
  }
  hipLaunchKernelGGL(k_loss_partial, dim3(kRedBlocks, nv), dim3(256), 0, s, (const double*)part,
                     lr, part2);
  GS_LAUNCHED("loss_partial");
  ImagePtrs im;
  for (int v = 0; v < nv; ++v) {
    im.x[v] = x[v];
    im.y[v] = y[v];
  }
  hipLaunchKernelGGL(k_sq_partial, dim3(kRedBlocks, nv), dim3(256), 0, s, im, lr, part3);
  GS_LAUNCHED("sq_partial");
  hipLaunchKernelGGL(k_metrics_final, dim3(nv), dim3(256), 0, s, (const double*)part2,
                     (const double*)part3, lr, out);
  GS_LAUNCHED("metrics_final");
  return GS_OK;
}

void loss_scratch_free(Ctx* ctx, LossScratch& ls) {
  buf_free(ctx, ls.gmap);
  buf_free(ctx, ls.part);
  if (ls.last_use != nullptr) (void)hipEventDestroy(ls.last_use);
  ls.last_use = nullptr;
}

}  // namespace isogs
