// Per-Gaussian stages: EWA projection + SH colour (forward) and the chain rule
// back to the parameters (backward).
//
// One thread per Gaussian loops over the frame's views, so the 236 B of
// parameters (SH degree 3) are read from HBM once per launch whatever the view
// count.  Geometry is evaluated in float64 with a fixed operation order (the
// library is built with -ffp-contract=off): the integer decisions that feed
// binning (near cull, radius, pixel and tile rectangle) and the float32 depth
// used in sort keys are then those of any IEEE float64 evaluation of the same
// formulas.  SH colour runs in float32.  Frames of at most four views (every
// form measured here) take kernels that stream the 48 SH coefficients one triple
// at a time and hold only per-view state, instead of holding the coefficients
// for the whole view loop (the batched four-view projection: 0.41 against
// 0.52 ms for 4M Gaussians, four instead of two waves per SIMD).
#include <type_traits>

#include "internal.h"

namespace isogs {
namespace {

constexpr double kLowpass = 0.3;  // EWA low-pass added to the 2-D covariance

// Real SH basis, degree <= 3, Condon-Shortley phase, m = -l..l.
constexpr float kK0 = 0.28209479177387814f;   // 1/(2 sqrt(pi))
constexpr float kK1 = 0.48860251190291992f;   // sqrt(3/(4 pi))
constexpr float kK2 = 1.09254843059207907f;   // sqrt(15/pi)/2
constexpr float kK3 = 0.31539156525252005f;   // sqrt(5/pi)/4
constexpr float kA3 = 0.59004358992664352f;   // sqrt(35/(2 pi))/4
constexpr float kB3 = 2.89061144264055405f;   // sqrt(105/pi)/2
constexpr float kC3 = 0.45704579946446572f;   // sqrt(21/(2 pi))/4
constexpr float kE3 = 0.37317633259011540f;   // sqrt(7/pi)/4

// Y_j of the real SH basis (degree <= 3, Condon-Shortley phase, m = -l..l) at a
// unit direction: the one definition of the basis polynomials.
template <int J>
__device__ inline float sh_value(float x, float y, float z) {
  if constexpr (J == 0) return kK0;
  else if constexpr (J == 1) return -kK1 * y;
  else if constexpr (J == 2) return kK1 * z;
  else if constexpr (J == 3) return -kK1 * x;
  else if constexpr (J == 4) return kK2 * x * y;
  else if constexpr (J == 5) return -kK2 * y * z;
  else if constexpr (J == 6) return kK3 * (2.f * (z * z) - (x * x) - (y * y));
  else if constexpr (J == 7) return -kK2 * x * z;
  else if constexpr (J == 8) return 0.5f * kK2 * ((x * x) - (y * y));
  else {
    const float xx = x * x, yy = y * y, zz = z * z;
    if constexpr (J == 9) return -kA3 * y * (3.f * xx - yy);
    else if constexpr (J == 10) return kB3 * x * y * z;
    else if constexpr (J == 11) return -kC3 * y * (4.f * zz - xx - yy);
    else if constexpr (J == 12) return kE3 * z * (2.f * zz - 3.f * xx - 3.f * yy);
    else if constexpr (J == 13) return -kC3 * x * (4.f * zz - xx - yy);
    else if constexpr (J == 14) return 0.5f * kB3 * z * (xx - yy);
    else return -kA3 * x * (xx - 3.f * yy);
  }
}

// Y[j] for every basis function of degree <= DEG.
template <int DEG, int J = 0>
__device__ inline void sh_basis(float x, float y, float z, float* Y) {
  if constexpr (J < (DEG + 1) * (DEG + 1)) {
    Y[J] = sh_value<J>(x, y, z);
    sh_basis<DEG, J + 1>(x, y, z, Y);
  }
}

// One basis function j at a unit direction: w grad Y_j added to g (each weight
// scaled once and the terms fused into multiply-adds: the backward takes no
// binning decision, so its rounding is free to differ from the forward's), and
// Y_j returned.  Summed over j in increasing order by sh_grad_w and by the
// coefficient-streaming colour backward alike.
struct Dir {
  float x, y, z;
};

template <int J>
__device__ inline float sh_term(const Dir& d, float w, float& gx, float& gy, float& gz) {
  const float x = d.x, y = d.y, z = d.z;
  if constexpr (J == 0) {
    return sh_value<J>(x, y, z);
  } else if constexpr (J == 1) {
    gy += -kK1 * w;
    return sh_value<J>(x, y, z);
  } else if constexpr (J == 2) {
    gz += kK1 * w;
    return sh_value<J>(x, y, z);
  } else if constexpr (J == 3) {
    gx += -kK1 * w;
    return sh_value<J>(x, y, z);
  } else if constexpr (J == 4) {
    const float t = kK2 * w;
    gx = fmaf(y, t, gx);
    gy = fmaf(x, t, gy);
    return sh_value<J>(x, y, z);
  } else if constexpr (J == 5) {
    const float t = kK2 * w;
    gy = fmaf(-z, t, gy);
    gz = fmaf(-y, t, gz);
    return sh_value<J>(x, y, z);
  } else if constexpr (J == 6) {
    const float t = 2.f * kK3 * w;
    gx = fmaf(-x, t, gx);
    gy = fmaf(-y, t, gy);
    gz = fmaf(2.f * z, t, gz);
    return sh_value<J>(x, y, z);
  } else if constexpr (J == 7) {
    const float t = kK2 * w;
    gx = fmaf(-z, t, gx);
    gz = fmaf(-x, t, gz);
    return sh_value<J>(x, y, z);
  } else if constexpr (J == 8) {
    const float t = kK2 * w;
    gx = fmaf(x, t, gx);
    gy = fmaf(-y, t, gy);
    return sh_value<J>(x, y, z);
  } else {
    const float xx = x * x, yy = y * y, zz = z * z;
    const float xy = x * y, yz = y * z, xz = x * z, dxy = xx - yy;
    if constexpr (J == 9) {
      const float t = kA3 * w;
      gx = fmaf(-6.f * xy, t, gx);
      gy = fmaf(-3.f * dxy, t, gy);
      return sh_value<J>(x, y, z);
    } else if constexpr (J == 10) {
      const float t = kB3 * w;
      gx = fmaf(yz, t, gx);
      gy = fmaf(xz, t, gy);
      gz = fmaf(xy, t, gz);
      return sh_value<J>(x, y, z);
    } else if constexpr (J == 11) {
      const float t = kC3 * w;
      gx = fmaf(2.f * xy, t, gx);
      gy = fmaf(-(4.f * zz - xx - 3.f * yy), t, gy);
      gz = fmaf(-8.f * yz, t, gz);
      return sh_value<J>(x, y, z);
    } else if constexpr (J == 12) {
      const float t = kE3 * w;
      gx = fmaf(-6.f * xz, t, gx);
      gy = fmaf(-6.f * yz, t, gy);
      gz = fmaf(6.f * zz - 3.f * xx - 3.f * yy, t, gz);
      return sh_value<J>(x, y, z);
    } else if constexpr (J == 13) {
      const float t = kC3 * w;
      gx = fmaf(-(4.f * zz - 3.f * xx - yy), t, gx);
      gy = fmaf(2.f * xy, t, gy);
      gz = fmaf(-8.f * xz, t, gz);
      return sh_value<J>(x, y, z);
    } else if constexpr (J == 14) {
      const float t = kB3 * w;
      gx = fmaf(xz, t, gx);
      gy = fmaf(-yz, t, gy);
      gz = fmaf(0.5f * dxy, t, gz);
      return sh_value<J>(x, y, z);
    } else {
      const float t = kA3 * w;
      gx = fmaf(-3.f * dxy, t, gx);
      gy = fmaf(6.f * xy, t, gy);
      return sh_value<J>(x, y, z);
    }
  }
}

// g = sum_j w[j] grad Y_j at the unit direction (x, y, z).
template <int DEG, int J = 0>
__device__ inline void sh_grad_w_acc(const Dir& d, const float* w, float& gx, float& gy, float& gz) {
  if constexpr (J < (DEG + 1) * (DEG + 1)) {
    (void)sh_term<J>(d, w[J], gx, gy, gz);
    sh_grad_w_acc<DEG, J + 1>(d, w, gx, gy, gz);
  }
}

template <int DEG>
__device__ inline void sh_grad_w(float x, float y, float z, const float* w, float& gx, float& gy,
                                 float& gz) {
  gx = gy = gz = 0.f;
  sh_grad_w_acc<DEG>(Dir{x, y, z}, w, gx, gy, gz);
}

// View-independent 3-D state of one Gaussian.
// Per-Gaussian state in precision F: float64 for the forward (its binning
// decisions must be those of any float64 evaluation), float32 for the
// backward, which takes no such decision.
template <typename F>
struct BodyT {
  F mu[3];
  F s[3];      // exp(log_scale)
  F qn[4];     // normalised quaternion (w, x, y, z)
  F qnorm;
  F Rq[9];     // rotation, row-major
  F Sig[9];    // 3-D covariance, row-major (symmetric)
};
using Body = BodyT<double>;

template <typename F>
__device__ inline void load_body(const ParamsDev& p, int i, BodyT<F>& b) {
  const int n = p.n;
  for (int k = 0; k < 3; ++k) {
    b.mu[k] = (F)p.means[k * n + i];
    b.s[k] = exp((F)p.log_scales[k * n + i]);
  }
  F q[4];
  for (int k = 0; k < 4; ++k) q[k] = (F)p.quats[k * n + i];
  b.qnorm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  if constexpr (sizeof(F) == 8) {
    for (int k = 0; k < 4; ++k) b.qn[k] = q[k] / b.qnorm;
  } else {
    const F iq = (F)1 / b.qnorm;
    for (int k = 0; k < 4; ++k) b.qn[k] = q[k] * iq;
  }
  const F w = b.qn[0], x = b.qn[1], y = b.qn[2], z = b.qn[3];
  F* R = b.Rq;
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
  F M[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) M[r * 3 + c] = R[r * 3 + c] * b.s[c];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      b.Sig[r * 3 + c] = M[r * 3 + 0] * M[c * 3 + 0] + M[r * 3 + 1] * M[c * 3 + 1] +
                         M[r * 3 + 2] * M[c * 3 + 2];
}

// Per-view projected state (R = double for the forward, whose binning
// decisions must be those of any float64 evaluation; float for the backward).
template <typename R>
struct ProjT {
  R t[3];
  R xz, yz, u, v, limx, limy;
  R J00, J02, J11, J12;
  R T0[3], T1[3];
  R S0[3], S1[3];  // Sigma3 T0, Sigma3 T1
  R a, b, c, det;
  R mx, my;
  int radius;
  int x0, y0, x1, y1;  // tile rectangle (inclusive); empty if !touched
  bool visible, touched;
};
using Proj = ProjT<double>;

// Camera-space mean, Jacobian and 2-D covariance (with the low-pass) of one view.
template <typename R>
__device__ inline void view_cov(const R* mu, const R* Sig, const CamDev& c, ProjT<R>& p) {
  const float* Rc = c.R;
  for (int r = 0; r < 3; ++r)
    p.t[r] = (R)Rc[r * 3 + 0] * mu[0] + (R)Rc[r * 3 + 1] * mu[1] + (R)Rc[r * 3 + 2] * mu[2] +
             (R)c.t[r];
  p.touched = false;
  p.visible = p.t[2] > (R)c.znear;
  const R tz = p.visible ? p.t[2] : R(1);
  const R fx = (R)c.fx, fy = (R)c.fy;
  if constexpr (sizeof(R) == 8) {
    // float64: the divisions of the definition (binning decisions follow them);
    // the guard-band limits, the same for every Gaussian, come with the camera
    p.limx = c.limx;
    p.limy = c.limy;
    p.xz = p.t[0] / tz;
    p.yz = p.t[1] / tz;
    p.u = fmin(fmax(p.xz, -p.limx), p.limx);
    p.v = fmin(fmax(p.yz, -p.limy), p.limy);
    p.J00 = fx / tz;
    p.J02 = -fx * p.u / tz;
    p.J11 = fy / tz;
    p.J12 = -fy * p.v / tz;
  } else {
    // float32 (gradients only): one hardware reciprocal of t_z (1 ulp) and products
    const R itz = __builtin_amdgcn_rcpf(tz);
    p.limx = R(kGuard) * (R(0.5) * (R)c.W * __builtin_amdgcn_rcpf(fx));
    p.limy = R(kGuard) * (R(0.5) * (R)c.H * __builtin_amdgcn_rcpf(fy));
    p.xz = p.t[0] * itz;
    p.yz = p.t[1] * itz;
    p.u = fmin(fmax(p.xz, -p.limx), p.limx);
    p.v = fmin(fmax(p.yz, -p.limy), p.limy);
    p.J00 = fx * itz;
    p.J02 = -fx * p.u * itz;
    p.J11 = fy * itz;
    p.J12 = -fy * p.v * itz;
  }
  for (int j = 0; j < 3; ++j) {
    p.T0[j] = p.J00 * (R)Rc[0 * 3 + j] + p.J02 * (R)Rc[2 * 3 + j];
    p.T1[j] = p.J11 * (R)Rc[1 * 3 + j] + p.J12 * (R)Rc[2 * 3 + j];
  }
  R* S0 = p.S0;
  R* S1 = p.S1;
  for (int r = 0; r < 3; ++r) {
    S0[r] = Sig[r * 3 + 0] * p.T0[0] + Sig[r * 3 + 1] * p.T0[1] + Sig[r * 3 + 2] * p.T0[2];
    S1[r] = Sig[r * 3 + 0] * p.T1[0] + Sig[r * 3 + 1] * p.T1[1] + Sig[r * 3 + 2] * p.T1[2];
  }
  p.a = p.T0[0] * S0[0] + p.T0[1] * S0[1] + p.T0[2] * S0[2] + R(kLowpass);
  p.b = p.T0[0] * S1[0] + p.T0[1] * S1[1] + p.T0[2] * S1[2];
  p.c = p.T1[0] * S1[0] + p.T1[1] * S1[1] + p.T1[2] * S1[2] + R(kLowpass);
  p.det = p.a * p.c - p.b * p.b;
  p.mx = fx * p.xz + (R)c.cx;
  p.my = fy * p.yz + (R)c.cy;
}

// view_cov plus the radius and the tile rectangle (the binning decisions).
__device__ inline void project_view(const Body& b, const CamDev& c, int tile, Proj& p) {
  view_cov(b.mu, b.Sig, c, p);
  p.radius = 0;
  if (!p.visible || !(p.det > 0)) return;
  const double half = 0.5 * (p.a - p.c);
  const double lmax = 0.5 * (p.a + p.c) + sqrt(half * half + p.b * p.b);
  const double r = ceil(3.0 * sqrt(fmax(lmax, 0.0)));
  // pixels whose centres lie in [m - r, m + r], clamped to the image
  double lox = ceil(p.mx - 0.5 - r), hix = floor(p.mx - 0.5 + r);
  double loy = ceil(p.my - 0.5 - r), hiy = floor(p.my - 0.5 + r);
  lox = fmax(lox, 0.0);
  loy = fmax(loy, 0.0);
  hix = fmin(hix, (double)(c.W - 1));
  hiy = fmin(hiy, (double)(c.H - 1));
  if (!(r > 0) || lox > hix || loy > hiy) return;
  p.radius = (int)r;
  p.x0 = (int)lox / tile;
  p.y0 = (int)loy / tile;
  p.x1 = (int)hix / tile;
  p.y1 = (int)hiy / tile;
  p.touched = true;
}

// Smallest fp16 not below x > 0 (bits); +inf past the largest finite value.
__device__ inline uint32_t half_bits_up(float x) {
  const _Float16 h = (_Float16)x;
  uint16_t b;
  __builtin_memcpy(&b, &h, 2);
  if ((float)h < x) ++b;  // positive halves order like their bit patterns
  return b;
}

// Half-widths of the axis-aligned box outside which alpha < 1/255 for certain,
// from the stored float32 conic and opacity: the ellipse power >= -ln(255 o)
// bounded by sqrt(c2 C / det) and sqrt(c2 A / det), widened by 1% + 0.01 px and
// rounded up to fp16 (x in the low half, y in the high).  Negative (-1) when
// the splat can never pass the alpha test.
__device__ inline uint32_t alpha_box_bits(float A, float B, float C, float o) {
  const float lim = o * 255.0f;
  // determinant in float64: the float32 conic of an elongated splat loses digits here
  const double det = (double)A * (double)C - (double)B * (double)B;
  if (!(lim >= 1.0f) || !(det > 0.0)) return 0xBC00BC00u;  // fp16 -1, -1
  const double c2 = 2.0 * ((double)logf(lim) + 1e-3);  // bound of dx^T Q dx, with margin
  // the square roots in float32: their relative error (~1e-7) is far inside the margin
  const double q = c2 / det;
  const float hw = sqrtf((float)(q * (double)C)) * 1.01f + 1e-2f;
  const float hh = sqrtf((float)(q * (double)A)) * 1.01f + 1e-2f;
  return half_bits_up(hw) | (half_bits_up(hh) << 16);
}

// Outputs of the projection forward, indexed by (view, Gaussian) entry.
struct FwdOut {
  float4* splat;
  uint2* rect;
  uint32_t* dkey;
  uint8_t* clampm;
  int32_t* radii;
};

// One (view, Gaussian) entry: tile rectangle, depth key and radius, and for a
// touched entry the clamp mask and splat record.  colour(rgb) gives the SH sum
// of each channel; the 0.5 offset and the clamp at zero are applied here.
template <class Colour>
__device__ inline void write_entry(const Body& b, const CamDev& c, int tile, size_t o,
                                   float opacity, const FwdOut& out, Colour colour) {
  Proj p;
  project_view(b, c, tile, p);
  if (out.radii != nullptr) out.radii[o] = p.radius;  // 0 unless touched
  if (!p.touched) {
    out.rect[o] = make_uint2(1u | (1u << 16), 0u);
    out.dkey[o] = 0xffffffffu;
    return;
  }
  const float depth = (float)p.t[2];
  out.rect[o] = make_uint2((uint32_t)p.x0 | ((uint32_t)p.y0 << 16),
                           (uint32_t)p.x1 | ((uint32_t)p.y1 << 16));
  out.dkey[o] = __float_as_uint(depth);
  float rgb[3];
  colour(rgb);
  uint32_t mask = 0;
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    float acc = rgb[ch] + 0.5f;
    if (acc < 0.f) {
      mask |= 1u << ch;
      acc = 0.f;
    }
    rgb[ch] = acc;
  }
  out.clampm[o] = (uint8_t)mask;
  const double fmx = floor(p.mx), fmy = floor(p.my);
  const double cmx = fmin(fmax(fmx, -1073741824.0), 1073741824.0);
  const double cmy = fmin(fmax(fmy, -1073741824.0), 1073741824.0);
  // conic = (c, -b, a) / det through one float64 reciprocal: within a float64 ulp of
  // the quotients, so the stored float32 values are the rounded quotients but for
  // rare ties of the double rounding (no binning decision reads them)
  const double idet = 1.0 / p.det;
  const float cA = (float)(p.c * idet), cB = (float)(-p.b * idet), cC = (float)(p.a * idet);
  out.splat[o * 3 + 0] = make_float4(cA, cB, cC, opacity);
  out.splat[o * 3 + 1] = make_float4(__int_as_float((int)cmx), __int_as_float((int)cmy),
                                     (float)(0.5 - (p.mx - cmx)), (float)(0.5 - (p.my - cmy)));
  out.splat[o * 3 + 2] =
      make_float4(rgb[0], rgb[1], rgb[2], __uint_as_float(alpha_box_bits(cA, cB, cC, opacity)));
}

constexpr int kShAheadFwd = 4;  // coefficient triples in flight ahead of the one in use

// rgb_v += sh[j] Y_j(d_v) for every view, coefficient triple by triple (the sum
// over j in increasing order, multiply then add, as in k_preprocess_fwd).
template <int DEG, int NV, int J>
__device__ inline void sh_colour_stream(const float* __restrict__ shc, int i, int n,
                                        const float (&dx)[NV], const float (&dy)[NV],
                                        const float (&dz)[NV], float (&rgb)[NV][3],
                                        float (&q)[kShAheadFwd][3]) {
  constexpr int NB = (DEG + 1) * (DEG + 1);
  if constexpr (J < NB) {
    const float s[3] = {q[J % kShAheadFwd][0], q[J % kShAheadFwd][1], q[J % kShAheadFwd][2]};
    if constexpr (J + kShAheadFwd < NB) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
        q[J % kShAheadFwd][c] = shc[(size_t)((J + kShAheadFwd) * 3 + c) * n + i];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const float Y = sh_value<J>(dx[v], dy[v], dz[v]);
#pragma unroll
      for (int c = 0; c < 3; ++c) rgb[v][c] += s[c] * Y;
    }
    sh_colour_stream<DEG, NV, J + 1>(shc, i, n, dx, dy, dz, rgb, q);
  }
}

// Forward for frames of at most four views: every view's colour first, with the
// SH coefficients streamed (only the views' colours held, not the 48
// coefficients, beside the float64 state), then the geometry view by view.  The
// same values as k_preprocess_fwd.
template <int DEG, int NV>
__global__ __launch_bounds__(256) void k_preprocess_fwd_few(ParamsDev prm, ViewTable vt,
                                                            float4* __restrict__ splat,
                                                            uint2* __restrict__ rect,
                                                            uint32_t* __restrict__ dkey,
                                                            uint8_t* __restrict__ clampm,
                                                            int32_t* __restrict__ radii,
                                                            const float* __restrict__ shc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = prm.n;
  if (i >= n) return;
  Body b;
  load_body(prm, i, b);
  const double logit = (double)prm.logits[i];
  const float opacity = (float)(1.0 / (1.0 + exp(-logit)));
  float dx[NV], dy[NV], dz[NV], rgb[NV][3];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const CamDev& c = vt.v[v];
    float x = (float)b.mu[0] - c.campos[0];
    float y = (float)b.mu[1] - c.campos[1];
    float z = (float)b.mu[2] - c.campos[2];
    const float inv = 1.0f / sqrtf(x * x + y * y + z * z);
    dx[v] = x * inv;
    dy[v] = y * inv;
    dz[v] = z * inv;
    rgb[v][0] = rgb[v][1] = rgb[v][2] = 0.f;
  }
  {
    float q[kShAheadFwd][3];
#pragma unroll
    for (int k = 0; k < kShAheadFwd && k < (DEG + 1) * (DEG + 1); ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) q[k][c] = shc[(size_t)(k * 3 + c) * n + i];
    sh_colour_stream<DEG, NV, 0>(shc, i, n, dx, dy, dz, rgb, q);
  }
  const FwdOut out{splat, rect, dkey, clampm, radii};
#pragma unroll
  for (int v = 0; v < NV; ++v)
    write_entry(b, vt.v[v], vt.tile, (size_t)v * n + i, opacity, out, [&](float (&col)[3]) {
      col[0] = rgb[v][0];
      col[1] = rgb[v][1];
      col[2] = rgb[v][2];
    });
}

template <int DEG>
__global__ __launch_bounds__(256) void k_preprocess_fwd(ParamsDev prm, ViewTable vt,
                                                        float4* __restrict__ splat,
                                                        uint2* __restrict__ rect,
                                                        uint32_t* __restrict__ dkey,
                                                        uint8_t* __restrict__ clampm,
                                                        int32_t* __restrict__ radii) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = prm.n;
  if (i >= n) return;
  Body b;
  load_body(prm, i, b);
  const double logit = (double)prm.logits[i];
  const float opacity = (float)(1.0 / (1.0 + exp(-logit)));
  constexpr int nb = (DEG + 1) * (DEG + 1);
  const FwdOut out{splat, rect, dkey, clampm, radii};
  for (int v = 0; v < vt.n; ++v) {
    const CamDev& c = vt.v[v];
    write_entry(b, c, vt.tile, (size_t)v * n + i, opacity, out, [&](float (&col)[3]) {
      // view-dependent colour
      float dx = (float)b.mu[0] - c.campos[0];
      float dy = (float)b.mu[1] - c.campos[1];
      float dz = (float)b.mu[2] - c.campos[2];
      const float inv = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
      dx *= inv;
      dy *= inv;
      dz *= inv;
      float Y[16];
      sh_basis<DEG>(dx, dy, dz, Y);
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        float acc = 0.f;
#pragma unroll
        for (int j = 0; j < nb; ++j) acc += prm.sh[(size_t)(j * 3 + ch) * n + i] * Y[j];
        col[ch] = acc;
      }
    });
  }
}

// Chain rule from the screen-space accumulators (9 per view) to the parameters.
// No bit-exact decision is taken here, so the geometry runs in float32.  It is
// split in two kernels, run side by side, so that each keeps few values live:
//  * geometry: per view, conic and mean2D gradients -> dL/dt (camera space) ->
//    dL/dmean, and dL/dSigma3 summed over the views; then the scale and
//    rotation gradients once from that sum, and the opacity gradient;
//  * colour: per view, dL/d(SH coefficients) and the gradient of the view
//    direction with respect to the mean (added to the geometry kernel's mean
//    gradient); it also clears the accumulators for the next pass.  Up to four
//    views it streams the coefficients one triple at a time (0.48 against
//    0.53 ms for one 2048^2 view of 4M Gaussians, 0.74 against 0.75 ms for the
//    four-view step beside the geometry kernel), beyond that it holds them.
// One view takes the same pair: a single kernel doing both parts holds the
// geometry and the 48 coefficients at once and ran slower (0.61 against
// 0.52 ms for 4M Gaussians).

// One view's geometric terms: the conic, mean2D and opacity sums (a0, a1.xy of
// the accumulator) -> dL/dmean (camera-space chain) and dL/dSigma3 (symmetrised,
// entries 00 01 02 11 12 22), added to g_mu and Gs; opacity sum added to g_op.
__device__ inline void geom_view(const float* mu, const float* Sig, const CamDev& c, float4 a0,
                                 float4 a1, float* g_mu, float* Gs, float& g_op) {
  ProjT<float> p;
  view_cov(mu, Sig, c, p);
  const float gmx = a0.x, gmy = a0.y, gA = a0.z, gB = a0.w, gC = a1.x;
  g_op += a1.y;
  // conic (A, B, C) = (c, -b, a) / det (det >= 0.09: the low-pass)
  const float iD = __builtin_amdgcn_rcpf(p.det);
  const float gD = -(gA * p.c - gB * p.b + gC * p.a) * iD * iD;
  const float ga = gC * iD + gD * p.c;
  const float gb = -gB * iD - 2.f * gD * p.b;
  const float gc = gA * iD + gD * p.a;
  // Sigma2 = T Sigma3 T^T: dL/dT rows, and G + G^T with
  // G = ga T0 T0^T + gb T0 T1^T + gc T1 T1^T
  float gT0[3], gT1[3];
  for (int r = 0; r < 3; ++r) {
    gT0[r] = 2.f * ga * p.S0[r] + gb * p.S1[r];
    gT1[r] = gb * p.S0[r] + 2.f * gc * p.S1[r];
  }
  {
    int k = 0;
    for (int r = 0; r < 3; ++r)
      for (int q = r; q < 3; ++q, ++k) {
        const float g1 = ga * p.T0[r] * p.T0[q] + gb * p.T0[r] * p.T1[q] + gc * p.T1[r] * p.T1[q];
        const float g2 = ga * p.T0[q] * p.T0[r] + gb * p.T0[q] * p.T1[r] + gc * p.T1[q] * p.T1[r];
        Gs[k] += g1 + g2;
      }
  }
  // T = J R  ->  dJ = dT R^T (only the four non-zero Jacobian entries matter)
  const float* R = c.R;
  float gJ00 = 0.f, gJ02 = 0.f, gJ11 = 0.f, gJ12 = 0.f;
  for (int k = 0; k < 3; ++k) {
    gJ00 += gT0[k] * R[0 * 3 + k];
    gJ02 += gT0[k] * R[2 * 3 + k];
    gJ11 += gT1[k] * R[1 * 3 + k];
    gJ12 += gT1[k] * R[2 * 3 + k];
  }
  const float tx = p.t[0], ty = p.t[1], tz = p.t[2];
  const float fx = c.fx, fy = c.fy;
  const float itz = __builtin_amdgcn_rcpf(tz), itz2 = itz * itz;
  float gt[3] = {0.f, 0.f, 0.f};
  gt[2] += gJ00 * (-fx * itz2) + gJ11 * (-fy * itz2) + gJ02 * (fx * p.u * itz2) +
           gJ12 * (fy * p.v * itz2);
  const float gu = gJ02 * (-fx * itz);
  const float gv = gJ12 * (-fy * itz);
  if (p.xz >= -p.limx && p.xz <= p.limx) {
    gt[0] += gu * itz;
    gt[2] += -gu * tx * itz2;
  }
  if (p.yz >= -p.limy && p.yz <= p.limy) {
    gt[1] += gv * itz;
    gt[2] += -gv * ty * itz2;
  }
  // mean2D
  gt[0] += gmx * fx * itz;
  gt[1] += gmy * fy * itz;
  gt[2] += -(gmx * fx * tx + gmy * fy * ty) * itz2;
  for (int k = 0; k < 3; ++k)
    g_mu[k] += R[0 * 3 + k] * gt[0] + R[1 * 3 + k] * gt[1] + R[2 * 3 + k] * gt[2];
}

// Scale and rotation gradients from the summed dL/dSigma3, and the opacity
// logit's from the summed opacity gradient (float32 body of Gaussian i).
__device__ inline void geom_finish(const ParamsDev& prm, int i, const float* Gs, float g_op,
                                   float* g_ls, float* g_q, float& g_logit) {
  BodyT<float> b;
  load_body(prm, i, b);
  const float G[9] = {Gs[0], Gs[1], Gs[2], Gs[1], Gs[3], Gs[4], Gs[2], Gs[4], Gs[5]};
  // Sigma3 = M M^T, M = Rq diag(s)
  float M[9];
  for (int r = 0; r < 3; ++r)
    for (int q = 0; q < 3; ++q) M[r * 3 + q] = b.Rq[r * 3 + q] * b.s[q];
  float gM[9];
  for (int r = 0; r < 3; ++r)
    for (int q = 0; q < 3; ++q)
      gM[r * 3 + q] = G[r * 3 + 0] * M[0 * 3 + q] + G[r * 3 + 1] * M[1 * 3 + q] +
                      G[r * 3 + 2] * M[2 * 3 + q];
  float gR[9];
  for (int r = 0; r < 3; ++r)
    for (int q = 0; q < 3; ++q) gR[r * 3 + q] = gM[r * 3 + q] * b.s[q];
  for (int q = 0; q < 3; ++q) {
    const float gsq = gM[0 * 3 + q] * b.Rq[0 * 3 + q] + gM[1 * 3 + q] * b.Rq[1 * 3 + q] +
                      gM[2 * 3 + q] * b.Rq[2 * 3 + q];
    g_ls[q] = gsq * b.s[q];
  }
  // rotation of the unit quaternion, entry by entry
  const float w = b.qn[0], x = b.qn[1], y = b.qn[2], z = b.qn[3];
  const float* g = gR;
  const float gw = 2 * (-z * g[1] + y * g[2] + z * g[3] - x * g[5] - y * g[6] + x * g[7]);
  const float gx = 2 * (y * g[1] + z * g[2] + y * g[3] - 2 * x * g[4] - w * g[5] + z * g[6] +
                        w * g[7] - 2 * x * g[8]);
  const float gy = 2 * (-2 * y * g[0] + x * g[1] + w * g[2] + x * g[3] + z * g[5] - w * g[6] +
                        z * g[7] - 2 * y * g[8]);
  const float gz = 2 * (-2 * z * g[0] - w * g[1] + x * g[2] + w * g[3] - 2 * z * g[4] +
                        y * g[5] + x * g[6] + y * g[7]);
  const float dot = w * gw + x * gx + y * gy + z * gz;
  const float iq = 1.f / b.qnorm;
  g_q[0] = (gw - w * dot) * iq;
  g_q[1] = (gx - x * dot) * iq;
  g_q[2] = (gy - y * dot) * iq;
  g_q[3] = (gz - z * dot) * iq;
  const float op = 1.f / (1.f + expf(-prm.logits[i]));
  g_logit = g_op * op * (1.f - op);
}

// Mean, Sigma3 (float32) of Gaussian i.
__device__ inline void geom_body(const ParamsDev& prm, int i, float* mu, float* Sig) {
  BodyT<float> b;
  load_body(prm, i, b);
  for (int k = 0; k < 3; ++k) mu[k] = b.mu[k];
  for (int k = 0; k < 9; ++k) Sig[k] = b.Sig[k];
}

__global__ __launch_bounds__(256) void k_preprocess_bwd_geom(ParamsDev prm, ViewTable vt,
                                                             float* __restrict__ accG,
                                                             GradsDev gout) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = prm.n;
  if (i >= n) return;
  float mu[3], Sig[9];
  bool loaded = false;
  float g_mu[3] = {0.f, 0.f, 0.f}, g_op = 0.f;
  float Gs[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int v = 0; v < vt.n; ++v) {
    // untouched (view, Gaussian) entries, and touched ones without gradient, are zero
    float4* a = reinterpret_cast<float4*>(accG + ((size_t)v * n + i) * kAccG);
    const float4 a0 = a[0], a1 = a[1];
    if (a0.x == 0.f && a0.y == 0.f && a0.z == 0.f && a0.w == 0.f && a1.x == 0.f && a1.y == 0.f)
      continue;
    // leave the accumulator cleared for the next backward pass
    if (!gout.keep_screen) {
      a[0] = make_float4(0.f, 0.f, 0.f, 0.f);
      a[1] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    if (!loaded) {
      geom_body(prm, i, mu, Sig);
      loaded = true;
    }
    geom_view(mu, Sig, vt.v[v], a0, a1, g_mu, Gs, g_op);
  }
  float g_ls[3] = {0.f, 0.f, 0.f}, g_q[4] = {0.f, 0.f, 0.f, 0.f}, g_logit = 0.f;
  if (loaded) geom_finish(prm, i, Gs, g_op, g_ls, g_q, g_logit);
  // write (or add) the gradients; untouched Gaussians get zeros
  const bool add = gout.accumulate != 0;
  auto put = [&](float* dst, float val) {
    if (add) {
      if (loaded) *dst += val;
    } else {
      *dst = val;
    }
  };
  for (int k = 0; k < 3; ++k) put(gout.means + (size_t)k * n + i, g_mu[k]);
  for (int k = 0; k < 3; ++k) put(gout.log_scales + (size_t)k * n + i, g_ls[k]);
  for (int k = 0; k < 4; ++k) put(gout.quats + (size_t)k * n + i, g_q[k]);
  put(gout.logits + i, g_logit);
}

// Colour part for frames of more than four views (k_preprocess_bwd_sh_few below
// takes the others); runs beside k_preprocess_bwd_geom (on another stream), writes its
// term of the mean gradient to gmu (added to the geometry kernel's by
// k_add_means once both are done) and clears every accumulator it finds non-zero.  All of
// the Gaussian's coefficients and their gradient sums stay in registers while
// the views are walked one at a time, so each view's basis is evaluated once,
// and its direction gradient is one weighted basis gradient: the weight of
// basis j is sum_c dL/dcolour_c sh[j][c].  The next view's colour sums and
// clamp mask are loaded while the current one is processed.
template <int DEG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_preprocess_bwd_sh(
    ParamsDev prm, ViewTable vt, float* __restrict__ accC, const uint8_t* __restrict__ clampm,
    GradsDev gout, float* __restrict__ gmu) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = prm.n;
  if (i >= n) return;
  constexpr int deg = DEG;
  constexpr int nb = (DEG + 1) * (DEG + 1);
  const bool add = gout.accumulate != 0;
  float4* const acc4 = reinterpret_cast<float4*>(accC);
  float4 a_next = acc4[i];
  uint32_t m_next = clampm[i];
  float mf[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) mf[k] = prm.means[(size_t)k * n + i];
  float sh[nb][3], gsh[nb][3];
#pragma unroll
  for (int j = 0; j < nb; ++j)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      sh[j][c] = prm.sh[(size_t)(j * 3 + c) * n + i];
      gsh[j][c] = 0.f;
    }
  float gmf[3] = {0.f, 0.f, 0.f};
  bool any_col = false;
#pragma unroll 1
  for (int v = 0; v < vt.n; ++v) {
    const float4 a0 = a_next;
    const uint32_t mask = m_next;
    if (v + 1 < vt.n) {
      const size_t on = (size_t)(v + 1) * n + i;
      a_next = acc4[on];
      m_next = clampm[on];
    }
    // untouched entries, and touched ones without gradient, are zero
    const bool col = a0.x != 0.f || a0.y != 0.f || a0.z != 0.f;
    if (__builtin_amdgcn_ballot_w64(col) == 0) continue;  // no lane of the wave has work
    if (col) {
      // cleared for the next pass
      if (!gout.keep_screen) acc4[(size_t)v * n + i] = make_float4(0.f, 0.f, 0.f, 0.f);
      any_col = true;
    }
    const float gr0 = (col && !(mask & 1u)) ? a0.x : 0.f;
    const float gr1 = (col && !(mask & 2u)) ? a0.y : 0.f;
    const float gr2 = (col && !(mask & 4u)) ? a0.z : 0.f;
    const CamDev& cam = vt.v[v];
    const float dx = mf[0] - cam.campos[0], dy = mf[1] - cam.campos[1],
                dz = mf[2] - cam.campos[2];
    const float inv = col ? 1.0f / sqrtf(dx * dx + dy * dy + dz * dz) : 0.f;
    const float x = dx * inv, y = dy * inv, z = dz * inv;
    float Y[16], w[16];
    sh_basis<DEG>(x, y, z, Y);
#pragma unroll
    for (int j = 0; j < nb; ++j) {
      gsh[j][0] = fmaf(Y[j], gr0, gsh[j][0]);
      gsh[j][1] = fmaf(Y[j], gr1, gsh[j][1]);
      gsh[j][2] = fmaf(Y[j], gr2, gsh[j][2]);
      w[j] = fmaf(gr2, sh[j][2], fmaf(gr1, sh[j][1], gr0 * sh[j][0]));
    }
    float gx, gy, gz;
    sh_grad_w<DEG>(x, y, z, w, gx, gy, gz);
    // through the normalisation d = (mu - campos) / |mu - campos|
    const float dot = gx * x + gy * y + gz * z;
    gmf[0] += (gx - x * dot) * inv;
    gmf[1] += (gy - y * dot) * inv;
    gmf[2] += (gz - z * dot) * inv;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) gmu[(size_t)k * n + i] = gmf[k];  // zero without colour gradient
  if (any_col) {
#pragma unroll
    for (int j = 0; j < nb; ++j)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float* dst = gout.sh + (size_t)(j * 3 + c) * n + i;
        if (add)
          *dst += gsh[j][c];
        else
          *dst = gsh[j][c];
      }
  } else if (!add) {
    for (int j = 0; j < nb * 3; ++j) gout.sh[(size_t)j * n + i] = 0.f;
  }
}

// Colour part for frames of at most four views, coefficient by coefficient:
// every view's direction and colour gradient are formed first, then each
// coefficient triple is read, its gradient (summed over the views) stored, and
// its term of every view's direction gradient added, so the coefficient and
// gradient streams are read and written throughout the kernel instead of all at
// its start and end, and only the views' state stays in registers.  The
// arithmetic, and its order, is that of k_preprocess_bwd_sh.
constexpr int kShAhead = 4;  // coefficient triples in flight ahead of the one in use

template <int DEG, int NV, int J>
__device__ inline void sh_stream_coef(const float* __restrict__ shc, int i, int n,
                                      const Dir (&d)[NV], const float (&gr)[NV][3],
                                      float (&g)[NV][3], bool any_col, bool add,
                                      float* __restrict__ gsh, float (&q)[kShAhead][3]) {
  constexpr int NB = (DEG + 1) * (DEG + 1);
  if constexpr (J < NB) {
    const float s[3] = {q[J % kShAhead][0], q[J % kShAhead][1], q[J % kShAhead][2]};
    if constexpr (J + kShAhead < NB) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
        q[J % kShAhead][c] = shc[(size_t)((J + kShAhead) * 3 + c) * n + i];
    }
    float gs[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const float w = fmaf(gr[v][2], s[2], fmaf(gr[v][1], s[1], gr[v][0] * s[0]));
      const float Y = sh_term<J>(d[v], w, g[v][0], g[v][1], g[v][2]);
#pragma unroll
      for (int c = 0; c < 3; ++c) gs[c] = fmaf(Y, gr[v][c], gs[c]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float* dst = gsh + (size_t)(J * 3 + c) * n + i;
      if (any_col) {
        if (add)
          *dst += gs[c];
        else
          *dst = gs[c];
      } else if (!add) {
        *dst = 0.f;
      }
    }
    sh_stream_coef<DEG, NV, J + 1>(shc, i, n, d, gr, g, any_col, add, gsh, q);
  }
}

template <int DEG, int NV>
__global__ __launch_bounds__(256) void k_preprocess_bwd_sh_few(ParamsDev prm, ViewTable vt,
                                                               float* __restrict__ accC,
                                                               const uint8_t* __restrict__ clampm,
                                                               GradsDev gout,
                                                               float* __restrict__ gmu,
                                                               const float* __restrict__ shc,
                                                               float* __restrict__ gsh) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = prm.n;
  if (i >= n) return;
  float4* const acc4 = reinterpret_cast<float4*>(accC);
  float mf[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) mf[k] = prm.means[(size_t)k * n + i];
  Dir d[NV];
  float inv[NV], gr[NV][3], g[NV][3];
  bool any_col = false;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const size_t o = (size_t)v * n + i;
    const float4 a0 = acc4[o];
    const uint32_t mask = clampm[o];
    // untouched entries, and touched ones without gradient, are zero
    const bool col = a0.x != 0.f || a0.y != 0.f || a0.z != 0.f;
    if (col) {
      if (!gout.keep_screen) acc4[o] = make_float4(0.f, 0.f, 0.f, 0.f);  // for the next pass
      any_col = true;
    }
    gr[v][0] = (col && !(mask & 1u)) ? a0.x : 0.f;
    gr[v][1] = (col && !(mask & 2u)) ? a0.y : 0.f;
    gr[v][2] = (col && !(mask & 4u)) ? a0.z : 0.f;
    const CamDev& cam = vt.v[v];
    const float dx = mf[0] - cam.campos[0], dy = mf[1] - cam.campos[1],
                dz = mf[2] - cam.campos[2];
    inv[v] = col ? 1.0f / sqrtf(dx * dx + dy * dy + dz * dz) : 0.f;
    d[v] = Dir{dx * inv[v], dy * inv[v], dz * inv[v]};
    g[v][0] = g[v][1] = g[v][2] = 0.f;
  }
  float q[kShAhead][3];
#pragma unroll
  for (int k = 0; k < kShAhead && k < (DEG + 1) * (DEG + 1); ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c) q[k][c] = shc[(size_t)(k * 3 + c) * n + i];
  sh_stream_coef<DEG, NV, 0>(shc, i, n, d, gr, g, any_col, gout.accumulate != 0, gsh, q);
  // through the normalisation d = (mu - campos) / |mu - campos|, summed over the views
  float gmf[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const float dot = g[v][0] * d[v].x + g[v][1] * d[v].y + g[v][2] * d[v].z;
    gmf[0] += (g[v][0] - d[v].x * dot) * inv[v];
    gmf[1] += (g[v][1] - d[v].y * dot) * inv[v];
    gmf[2] += (g[v][2] - d[v].z * dot) * inv[v];
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) gmu[(size_t)k * n + i] = gmf[k];  // zero without colour gradient
}

// means gradient += the colour kernel's term (after both backward kernels)
__global__ __launch_bounds__(256) void k_add_means(float* __restrict__ means,
                                                   const float* __restrict__ gmu, int n3) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n3) means[i] += gmu[i];
}

}  // namespace

gs_status launch_preprocess_fwd(const ParamsDev& p, const ViewTable& vt, Frame& f,
                                hipStream_t s, size_t base) {
  const int blocks = (int)((p.n + 255) / 256);
  auto* sp = (float4*)f.splat.p + 3 * base;
  auto* rc = (uint2*)f.rect.p + base;
  auto* dk = (uint32_t*)f.dkey.p + base;
  auto* cm = (uint8_t*)f.clampm.p + base;
  auto* rd = f.keep_radii ? (int32_t*)f.radii.p + base : nullptr;
  auto few = [&](auto deg) {
    constexpr int D = decltype(deg)::value;
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, s, p, vt, sp, rc, dk, cm, rd,
                         (const float*)p.sh);
    };
    switch (vt.n) {
      case 1: go(k_preprocess_fwd_few<D, 1>); break;
      case 2: go(k_preprocess_fwd_few<D, 2>); break;
      case 3: go(k_preprocess_fwd_few<D, 3>); break;
      default: go(k_preprocess_fwd_few<D, 4>); break;
    }
  };
  if (vt.n >= 1 && vt.n <= 4) {
    switch (p.sh_degree) {
      case 0: few(std::integral_constant<int, 0>{}); break;
      case 1: few(std::integral_constant<int, 1>{}); break;
      case 2: few(std::integral_constant<int, 2>{}); break;
      default: few(std::integral_constant<int, 3>{}); break;
    }
  } else {
    switch (p.sh_degree) {
      case 0: hipLaunchKernelGGL(k_preprocess_fwd<0>, dim3(blocks), dim3(256), 0, s, p, vt, sp, rc, dk, cm, rd); break;
      case 1: hipLaunchKernelGGL(k_preprocess_fwd<1>, dim3(blocks), dim3(256), 0, s, p, vt, sp, rc, dk, cm, rd); break;
      case 2: hipLaunchKernelGGL(k_preprocess_fwd<2>, dim3(blocks), dim3(256), 0, s, p, vt, sp, rc, dk, cm, rd); break;
      default: hipLaunchKernelGGL(k_preprocess_fwd<3>, dim3(blocks), dim3(256), 0, s, p, vt, sp, rc, dk, cm, rd); break;
    }
  }
  GS_LAUNCHED("preprocess_fwd");
  return GS_OK;
}

gs_status launch_preprocess_bwd(const ParamsDev& p, const ViewTable& vt, Frame& f,
                                const GradsDev& g, hipStream_t s) {
  const int blocks = (int)((p.n + 255) / 256);
  auto* accG = (float*)f.acc.p;
  auto* accC = accG + (size_t)f.views * (size_t)f.n * kAccG;
  auto* cm = (const uint8_t*)f.clampm.p;
  // the geometry kernel (instruction-bound) on the frame's side stream, the colour
  // kernel (memory-bound) on s, joined before the colour kernel's mean term is added
  float* gmu = (float*)f.gmu.p;
  if (gmu == nullptr || f.side == nullptr) {
    set_error("internal: the frame has no side stream / mean scratch for %d views", vt.n);
    return GS_ERR_INVALID;
  }
  GS_HIP(hipEventRecord(f.fork_ev, s));
  GS_HIP(hipStreamWaitEvent(f.side, f.fork_ev, 0));
  hipLaunchKernelGGL(k_preprocess_bwd_geom, dim3(blocks), dim3(256), 0, f.side, p, vt, accG, g);
  GS_LAUNCHED("preprocess_bwd_geom");
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, s, p, vt, accC, cm, g, gmu);
  };
  // the coefficient and gradient arrays are distinct buffers (restrict
  // parameters: the coefficient loads may be scheduled ahead of gradient stores)
  auto go_few = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, s, p, vt, accC, cm, g, gmu,
                       (const float*)p.sh, g.sh);
  };
  auto few = [&](auto deg) {
    constexpr int D = decltype(deg)::value;
    switch (vt.n) {
      case 1: go_few(k_preprocess_bwd_sh_few<D, 1>); break;
      case 2: go_few(k_preprocess_bwd_sh_few<D, 2>); break;
      case 3: go_few(k_preprocess_bwd_sh_few<D, 3>); break;
      default: go_few(k_preprocess_bwd_sh_few<D, 4>); break;
    }
  };
  if (vt.n <= 4) {
    switch (p.sh_degree) {
      case 0: few(std::integral_constant<int, 0>{}); break;
      case 1: few(std::integral_constant<int, 1>{}); break;
      case 2: few(std::integral_constant<int, 2>{}); break;
      default: few(std::integral_constant<int, 3>{}); break;
    }
  } else {
    switch (p.sh_degree) {
      case 0: go(k_preprocess_bwd_sh<0>); break;
      case 1: go(k_preprocess_bwd_sh<1>); break;
      case 2: go(k_preprocess_bwd_sh<2>); break;
      default: go(k_preprocess_bwd_sh<3>); break;
    }
  }
  GS_LAUNCHED("preprocess_bwd_sh");
  GS_HIP(hipEventRecord(f.join_ev, f.side));
  GS_HIP(hipStreamWaitEvent(s, f.join_ev, 0));
  const int n3 = 3 * p.n;
  hipLaunchKernelGGL(k_add_means, dim3((n3 + 255) / 256), dim3(256), 0, s, g.means, gmu, n3);
  GS_LAUNCHED("add_means");
  return GS_OK;
}

}  // namespace isogs

// ------------------------------------------------------------------ init
// Gaussians from isosurface points.  Random draws come from Philox4x32-10
// (Salmon et al., "Parallel random numbers: as easy as 1, 2, 3", SC'11) keyed
// by the seed, with counter (Gaussian index, stream, block, 0):
//   stream 0: three uniforms for the log-scales;
//   stream 1: four normals (two Box-Muller pairs) for the quaternion;
//   stream 2, block b: normals 4b..4b+3 of the SH coefficients (row-major).
// Uniform u = (x >> 8) 2^-24; Box-Muller on (a, b):
//   r = sqrt(-2 ln(((a >> 8) + 0.5) 2^-24)), theta = 2 pi (b >> 8) 2^-24,
//   normals (r cos theta, r sin theta).
namespace isogs {
namespace {

__device__ inline float u24(uint32_t x) { return (float)(x >> 8) * (1.0f / 16777216.0f); }

__device__ inline void box_muller(uint32_t a, uint32_t b, float& z0, float& z1) {
  const float ua = ((float)(a >> 8) + 0.5f) * (1.0f / 16777216.0f);
  const float r = sqrtf(-2.0f * logf(ua));
  const float th = 6.283185307179586f * u24(b);
  z0 = r * cosf(th);
  z1 = r * sinf(th);
}

__global__ __launch_bounds__(256) void k_init_points(const float* __restrict__ xyz, int n,
                                                     gs_init_opts o, uint32_t k0, uint32_t k1,
                                                     gs_params out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int k = 0; k < 3; ++k) out.means[(size_t)k * n + i] = xyz[(size_t)k * n + i];
  uint32_t c[4] = {(uint32_t)i, 0u, 0u, 0u};
  philox4x32_10(c, k0, k1);
  const bool ranged = o.log_scale_lo < o.log_scale_hi;
  for (int k = 0; k < 3; ++k) {
    const float u = u24(c[k]);
    const float ls = ranged ? o.log_scale_lo + (o.log_scale_hi - o.log_scale_lo) * u
                            : o.log_scale + o.log_scale_jitter * (2.0f * u - 1.0f);
    out.log_scales[(size_t)k * n + i] = ls;
  }
  float q[4] = {1.f, 0.f, 0.f, 0.f};
  if (o.random_quats) {
    uint32_t d[4] = {(uint32_t)i, 1u, 0u, 0u};
    philox4x32_10(d, k0, k1);
    box_muller(d[0], d[1], q[0], q[1]);
    box_muller(d[2], d[3], q[2], q[3]);
    const float inv = 1.0f / sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int k = 0; k < 4; ++k) q[k] *= inv;
  }
  for (int k = 0; k < 4; ++k) out.quats[(size_t)k * n + i] = q[k];
  out.opacity_logits[i] = o.opacity_logit;
  const int rows = (out.sh_degree + 1) * (out.sh_degree + 1) * 3;
  for (int b = 0; b * 4 < rows; ++b) {
    float z[4] = {0.f, 0.f, 0.f, 0.f};
    if (o.sh_std > 0.f) {
      uint32_t d[4] = {(uint32_t)i, 2u, (uint32_t)b, 0u};
      philox4x32_10(d, k0, k1);
      box_muller(d[0], d[1], z[0], z[1]);
      box_muller(d[2], d[3], z[2], z[3]);
    }
    for (int k = 0; k < 4 && b * 4 + k < rows; ++k)
      out.sh[(size_t)(b * 4 + k) * n + i] = o.sh_std * z[k];
  }
}

}  // namespace

gs_status launch_init_points(const float* xyz, int64_t n, const gs_init_opts& o, uint64_t seed,
                             gs_params out, hipStream_t s) {
  hipLaunchKernelGGL(k_init_points, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, xyz,
                     (int)n, o, (uint32_t)seed, (uint32_t)(seed >> 32), out);
  GS_LAUNCHED("init_points");
  return GS_OK;
}

}  // namespace isogs
