// Per-Gaussian stages: EWA projection + SH colour (forward) and the chain rule
// back to the parameters (backward).
//
// One thread per Gaussian loops over the frame's views, so the 236 B of
// parameters (SH degree 3) are read from HBM once per launch whatever the view
// count.  Geometry is evaluated in float64 with a fixed operation order (the
// library is built with -ffp-contract=off): the integer decisions that feed
// binning (near cull, radius, pixel and tile rectangle) and the float32 depth
// used in sort keys are then those of any IEEE float64 evaluation of the same
// formulas.  SH colour runs in float32.
#include "internal.h"

namespace isogs {
namespace {

constexpr double kLowpass = 0.3;  // EWA low-pass added to the 2-D covariance
constexpr double kGuard = 1.3;    // guard band on t_x/t_z, t_y/t_z for the Jacobian

// Real SH basis, degree <= 3, Condon-Shortley phase, m = -l..l.
constexpr float kK0 = 0.28209479177387814f;   // 1/(2 sqrt(pi))
constexpr float kK1 = 0.48860251190291992f;   // sqrt(3/(4 pi))
constexpr float kK2 = 1.09254843059207907f;   // sqrt(15/pi)/2
constexpr float kK3 = 0.31539156525252005f;   // sqrt(5/pi)/4
constexpr float kA3 = 0.59004358992664352f;   // sqrt(35/(2 pi))/4
constexpr float kB3 = 2.89061144264055405f;   // sqrt(105/pi)/2
constexpr float kC3 = 0.45704579946446572f;   // sqrt(21/(2 pi))/4
constexpr float kE3 = 0.37317633259011540f;   // sqrt(7/pi)/4

__device__ inline void sh_basis(float x, float y, float z, int deg, float* Y) {
  Y[0] = kK0;
  if (deg < 1) return;
  Y[1] = -kK1 * y;
  Y[2] = kK1 * z;
  Y[3] = -kK1 * x;
  if (deg < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[4] = kK2 * x * y;
  Y[5] = -kK2 * y * z;
  Y[6] = kK3 * (2.f * zz - xx - yy);
  Y[7] = -kK2 * x * z;
  Y[8] = 0.5f * kK2 * (xx - yy);
  if (deg < 3) return;
  Y[9] = -kA3 * y * (3.f * xx - yy);
  Y[10] = kB3 * x * y * z;
  Y[11] = -kC3 * y * (4.f * zz - xx - yy);
  Y[12] = kE3 * z * (2.f * zz - 3.f * xx - 3.f * yy);
  Y[13] = -kC3 * x * (4.f * zz - xx - yy);
  Y[14] = 0.5f * kB3 * z * (xx - yy);
  Y[15] = -kA3 * x * (xx - 3.f * yy);
}

// d/d(x, y, z) of each basis polynomial, accumulated against weights w[j]:
// g += sum_j w[j] * grad Y_j.
__device__ inline void sh_basis_grad_dot(float x, float y, float z, int deg, const float* w,
                                         float& gx, float& gy, float& gz) {
  if (deg < 1) return;
  gy += -kK1 * w[1];
  gz += kK1 * w[2];
  gx += -kK1 * w[3];
  if (deg < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  gx += kK2 * y * w[4];
  gy += kK2 * x * w[4];
  gy += -kK2 * z * w[5];
  gz += -kK2 * y * w[5];
  gx += -2.f * kK3 * x * w[6];
  gy += -2.f * kK3 * y * w[6];
  gz += 4.f * kK3 * z * w[6];
  gx += -kK2 * z * w[7];
  gz += -kK2 * x * w[7];
  gx += kK2 * x * w[8];
  gy += -kK2 * y * w[8];
  if (deg < 3) return;
  gx += -kA3 * 6.f * x * y * w[9];
  gy += -kA3 * (3.f * xx - 3.f * yy) * w[9];
  gx += kB3 * y * z * w[10];
  gy += kB3 * x * z * w[10];
  gz += kB3 * x * y * w[10];
  gx += kC3 * 2.f * x * y * w[11];
  gy += -kC3 * (4.f * zz - xx - 3.f * yy) * w[11];
  gz += -kC3 * 8.f * y * z * w[11];
  gx += -kE3 * 6.f * x * z * w[12];
  gy += -kE3 * 6.f * y * z * w[12];
  gz += kE3 * (6.f * zz - 3.f * xx - 3.f * yy) * w[12];
  gx += -kC3 * (4.f * zz - 3.f * xx - yy) * w[13];
  gy += kC3 * 2.f * x * y * w[13];
  gz += -kC3 * 8.f * x * z * w[13];
  gx += kB3 * x * z * w[14];
  gy += -kB3 * y * z * w[14];
  gz += 0.5f * kB3 * (xx - yy) * w[14];
  gx += -kA3 * (3.f * xx - 3.f * yy) * w[15];
  gy += kA3 * 6.f * x * y * w[15];
}

// View-independent 3-D state of one Gaussian.
struct Body {
  double mu[3];
  double s[3];      // exp(log_scale)
  double qn[4];     // normalised quaternion (w, x, y, z)
  double qnorm;
  double Rq[9];     // rotation, row-major
  double Sig[9];    // 3-D covariance, row-major (symmetric)
};

__device__ inline void load_body(const ParamsDev& p, int i, Body& b) {
  const int n = p.n;
  for (int k = 0; k < 3; ++k) {
    b.mu[k] = (double)p.means[k * n + i];
    b.s[k] = exp((double)p.log_scales[k * n + i]);
  }
  double q[4];
  for (int k = 0; k < 4; ++k) q[k] = (double)p.quats[k * n + i];
  b.qnorm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int k = 0; k < 4; ++k) b.qn[k] = q[k] / b.qnorm;
  const double w = b.qn[0], x = b.qn[1], y = b.qn[2], z = b.qn[3];
  double* R = b.Rq;
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
  double M[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) M[r * 3 + c] = R[r * 3 + c] * b.s[c];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      b.Sig[r * 3 + c] = M[r * 3 + 0] * M[c * 3 + 0] + M[r * 3 + 1] * M[c * 3 + 1] +
                         M[r * 3 + 2] * M[c * 3 + 2];
}

// Per-view projected state.
struct Proj {
  double t[3];
  double xz, yz, u, v, limx, limy;
  double J00, J02, J11, J12;
  double T0[3], T1[3];
  double S0[3], S1[3];  // Sigma3 T0, Sigma3 T1
  double a, b, c, det;
  double mx, my;
  int radius;
  int x0, y0, x1, y1;  // tile rectangle (inclusive); empty if !touched
  bool visible, touched;
};

// Camera-space mean, Jacobian and 2-D covariance (with the low-pass) of one view.
__device__ inline void view_cov(const double* mu, const double* Sig, const CamDev& c, Proj& p) {
  const float* R = c.R;
  for (int r = 0; r < 3; ++r)
    p.t[r] = (double)R[r * 3 + 0] * mu[0] + (double)R[r * 3 + 1] * mu[1] +
             (double)R[r * 3 + 2] * mu[2] + (double)c.t[r];
  p.touched = false;
  p.visible = p.t[2] > (double)c.znear;
  const double tz = p.visible ? p.t[2] : 1.0;
  const double fx = c.fx, fy = c.fy;
  p.limx = kGuard * (0.5 * (double)c.W / fx);
  p.limy = kGuard * (0.5 * (double)c.H / fy);
  p.xz = p.t[0] / tz;
  p.yz = p.t[1] / tz;
  p.u = fmin(fmax(p.xz, -p.limx), p.limx);
  p.v = fmin(fmax(p.yz, -p.limy), p.limy);
  p.J00 = fx / tz;
  p.J02 = -fx * p.u / tz;
  p.J11 = fy / tz;
  p.J12 = -fy * p.v / tz;
  for (int j = 0; j < 3; ++j) {
    p.T0[j] = p.J00 * (double)R[0 * 3 + j] + p.J02 * (double)R[2 * 3 + j];
    p.T1[j] = p.J11 * (double)R[1 * 3 + j] + p.J12 * (double)R[2 * 3 + j];
  }
  double* S0 = p.S0;
  double* S1 = p.S1;
  for (int r = 0; r < 3; ++r) {
    S0[r] = Sig[r * 3 + 0] * p.T0[0] + Sig[r * 3 + 1] * p.T0[1] + Sig[r * 3 + 2] * p.T0[2];
    S1[r] = Sig[r * 3 + 0] * p.T1[0] + Sig[r * 3 + 1] * p.T1[1] + Sig[r * 3 + 2] * p.T1[2];
  }
  p.a = p.T0[0] * S0[0] + p.T0[1] * S0[1] + p.T0[2] * S0[2] + kLowpass;
  p.b = p.T0[0] * S1[0] + p.T0[1] * S1[1] + p.T0[2] * S1[2];
  p.c = p.T1[0] * S1[0] + p.T1[1] * S1[1] + p.T1[2] * S1[2] + kLowpass;
  p.det = p.a * p.c - p.b * p.b;
  p.mx = fx * p.xz + (double)c.cx;
  p.my = fy * p.yz + (double)c.cy;
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
  const float hw = (float)(sqrt(c2 * (double)C / det) * 1.01 + 1e-2);
  const float hh = (float)(sqrt(c2 * (double)A / det) * 1.01 + 1e-2);
  return half_bits_up(hw) | (half_bits_up(hh) << 16);
}

template <int DEG>
__global__ __launch_bounds__(256) void k_preprocess_fwd(ParamsDev prm, ViewTable vt,
                                                        float4* __restrict__ splat,
                                                        uint2* __restrict__ rect,
                                                        uint32_t* __restrict__ dkey,
                                                        uint8_t* __restrict__ clampm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = prm.n;
  if (i >= n) return;
  Body b;
  load_body(prm, i, b);
  const double logit = (double)prm.logits[i];
  const float opacity = (float)(1.0 / (1.0 + exp(-logit)));
  constexpr int deg = DEG;
  constexpr int nb = (DEG + 1) * (DEG + 1);
  for (int v = 0; v < vt.n; ++v) {
    const CamDev& c = vt.v[v];
    Proj p;
    project_view(b, c, vt.tile, p);
    const size_t o = (size_t)v * n + i;
    if (!p.touched) {
      rect[o] = make_uint2(1u | (1u << 16), 0u);
      dkey[o] = 0xffffffffu;
      continue;
    }
    const float depth = (float)p.t[2];
    rect[o] = make_uint2((uint32_t)p.x0 | ((uint32_t)p.y0 << 16),
                         (uint32_t)p.x1 | ((uint32_t)p.y1 << 16));
    dkey[o] = __float_as_uint(depth);
    // view-dependent colour
    float dx = (float)b.mu[0] - c.campos[0];
    float dy = (float)b.mu[1] - c.campos[1];
    float dz = (float)b.mu[2] - c.campos[2];
    const float inv = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
    dx *= inv;
    dy *= inv;
    dz *= inv;
    float Y[16];
    sh_basis(dx, dy, dz, deg, Y);
    float rgb[3];
    uint32_t mask = 0;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      float acc = 0.f;
#pragma unroll
      for (int j = 0; j < nb; ++j) acc += prm.sh[(size_t)(j * 3 + ch) * n + i] * Y[j];
      acc += 0.5f;
      if (acc < 0.f) {
        mask |= 1u << ch;
        acc = 0.f;
      }
      rgb[ch] = acc;
    }
    clampm[o] = (uint8_t)mask;
    const double fmx = floor(p.mx), fmy = floor(p.my);
    const double cmx = fmin(fmax(fmx, -1073741824.0), 1073741824.0);
    const double cmy = fmin(fmax(fmy, -1073741824.0), 1073741824.0);
    const float cA = (float)(p.c / p.det), cB = (float)(-p.b / p.det), cC = (float)(p.a / p.det);
    splat[o * 3 + 0] = make_float4(cA, cB, cC, opacity);
    splat[o * 3 + 1] = make_float4(__int_as_float((int)cmx), __int_as_float((int)cmy),
                                   (float)(0.5 - (p.mx - cmx)), (float)(0.5 - (p.my - cmy)));
    splat[o * 3 + 2] =
        make_float4(rgb[0], rgb[1], rgb[2], __uint_as_float(alpha_box_bits(cA, cB, cC, opacity)));
  }
}

// Chain rule from the screen-space accumulators (9 per view) to the parameters.
//
// Three phases keep few values live at a time:
//  1. geometry, float64, per view: conic and mean2D gradients -> dL/dt (camera
//     space) -> dL/dmean, and dL/dSigma3 summed over the views (dL/dSigma3 is
//     all that the scale and rotation gradients need, so their chain runs once);
//  2. SH colour, float32, per view: dL/d(SH coefficients) and the gradient of
//     the view direction with respect to the mean; the accumulators are
//     cleared for the next pass here;
//  3. scale and rotation from the summed dL/dSigma3.
template <int DEG>
__global__ __launch_bounds__(256) void k_preprocess_bwd(ParamsDev prm, ViewTable vt,
                                                        float* __restrict__ acc,
                                                        const uint2* __restrict__ rect,
                                                        const uint8_t* __restrict__ clampm,
                                                        GradsDev gout) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = prm.n;
  if (i >= n) return;
  constexpr int deg = DEG;
  constexpr int nb = (DEG + 1) * (DEG + 1);

  // ---- 1. geometry
  double mu[3], Sig[9];
  bool loaded = false, any = false;
  double g_mu[3] = {0, 0, 0}, g_op = 0;
  double Gs[6] = {0, 0, 0, 0, 0, 0};  // dL/dSigma3 (symmetrised): 00 01 02 11 12 22
  for (int v = 0; v < vt.n; ++v) {
    const size_t o = (size_t)v * n + i;
    const uint2 rc = rect[o];
    if ((rc.y & 0xffffu) < (rc.x & 0xffffu)) continue;  // untouched in this view
    const float4* a = reinterpret_cast<const float4*>(acc + o * kAccStride);
    const float4 a0 = a[0], a1 = a[1];
    if (a0.x == 0.f && a0.y == 0.f && a0.z == 0.f && a0.w == 0.f && a1.x == 0.f && a1.y == 0.f)
      continue;
    if (!loaded) {
      Body b;
      load_body(prm, i, b);
      for (int k = 0; k < 3; ++k) mu[k] = b.mu[k];
      for (int k = 0; k < 9; ++k) Sig[k] = b.Sig[k];
      loaded = true;
    }
    const CamDev& c = vt.v[v];
    Proj p;
    view_cov(mu, Sig, c, p);
    const double gmx = a0.x, gmy = a0.y, gA = a0.z, gB = a0.w, gC = a1.x;
    g_op += a1.y;
    // conic (A, B, C) = (c, -b, a) / det
    const double D = p.det;
    const double gD = -(gA * p.c - gB * p.b + gC * p.a) / (D * D);
    const double ga = gC / D + gD * p.c;
    const double gb = -gB / D - 2.0 * gD * p.b;
    const double gc = gA / D + gD * p.a;
    // Sigma2 = T Sigma3 T^T: dL/dT rows, and G + G^T with
    // G = ga T0 T0^T + gb T0 T1^T + gc T1 T1^T
    double gT0[3], gT1[3];
    for (int r = 0; r < 3; ++r) {
      gT0[r] = 2.0 * ga * p.S0[r] + gb * p.S1[r];
      gT1[r] = gb * p.S0[r] + 2.0 * gc * p.S1[r];
    }
    {
      int k = 0;
      for (int r = 0; r < 3; ++r)
        for (int q = r; q < 3; ++q, ++k) {
          const double g1 = ga * p.T0[r] * p.T0[q] + gb * p.T0[r] * p.T1[q] + gc * p.T1[r] * p.T1[q];
          const double g2 = ga * p.T0[q] * p.T0[r] + gb * p.T0[q] * p.T1[r] + gc * p.T1[q] * p.T1[r];
          Gs[k] += g1 + g2;
        }
    }
    // T = J R  ->  dJ = dT R^T (only the four non-zero Jacobian entries matter)
    const float* R = c.R;
    double gJ00 = 0, gJ02 = 0, gJ11 = 0, gJ12 = 0;
    for (int k = 0; k < 3; ++k) {
      gJ00 += gT0[k] * (double)R[0 * 3 + k];
      gJ02 += gT0[k] * (double)R[2 * 3 + k];
      gJ11 += gT1[k] * (double)R[1 * 3 + k];
      gJ12 += gT1[k] * (double)R[2 * 3 + k];
    }
    const double tx = p.t[0], ty = p.t[1], tz = p.t[2];
    const double fx = c.fx, fy = c.fy;
    double gt[3] = {0, 0, 0};
    gt[2] += gJ00 * (-fx / (tz * tz)) + gJ11 * (-fy / (tz * tz)) + gJ02 * (fx * p.u / (tz * tz)) +
             gJ12 * (fy * p.v / (tz * tz));
    const double gu = gJ02 * (-fx / tz);
    const double gv = gJ12 * (-fy / tz);
    if (p.xz >= -p.limx && p.xz <= p.limx) {
      gt[0] += gu / tz;
      gt[2] += -gu * tx / (tz * tz);
    }
    if (p.yz >= -p.limy && p.yz <= p.limy) {
      gt[1] += gv / tz;
      gt[2] += -gv * ty / (tz * tz);
    }
    // mean2D
    gt[0] += gmx * fx / tz;
    gt[1] += gmy * fy / tz;
    gt[2] += -(gmx * fx * tx + gmy * fy * ty) / (tz * tz);
    for (int k = 0; k < 3; ++k)
      g_mu[k] += (double)R[0 * 3 + k] * gt[0] + (double)R[1 * 3 + k] * gt[1] +
                 (double)R[2 * 3 + k] * gt[2];
  }

  // ---- 2. SH colour (float32); clears the accumulators
  float g_sh[nb * 3];
#pragma unroll
  for (int j = 0; j < nb * 3; ++j) g_sh[j] = 0.f;
  float gmf[3] = {0.f, 0.f, 0.f};
  float mf[3] = {0.f, 0.f, 0.f};
  bool mf_loaded = false;
  for (int v = 0; v < vt.n; ++v) {
    const size_t o = (size_t)v * n + i;
    const uint2 rc = rect[o];
    if ((rc.y & 0xffffu) < (rc.x & 0xffffu)) continue;
    float4* a = reinterpret_cast<float4*>(acc + o * kAccStride);
    const float4 a0 = a[0], a1 = a[1], a2 = a[2];
    const bool geo = a0.x != 0.f || a0.y != 0.f || a0.z != 0.f || a0.w != 0.f || a1.x != 0.f ||
                     a1.y != 0.f;
    const bool col = a1.z != 0.f || a1.w != 0.f || a2.x != 0.f;
    if (!geo && !col) continue;
    // leave the accumulator cleared for the next backward pass
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
    a[0] = zero4;
    a[1] = zero4;
    a[2] = zero4;
    any = true;
    if (!col) continue;
    const uint32_t mask = clampm[o];
    const float grgb[3] = {(mask & 1u) ? 0.f : a1.z, (mask & 2u) ? 0.f : a1.w,
                           (mask & 4u) ? 0.f : a2.x};
    if (!mf_loaded) {
      for (int k = 0; k < 3; ++k) mf[k] = (float)(double)prm.means[k * n + i];
      mf_loaded = true;
    }
    const CamDev& c = vt.v[v];
    float dx = mf[0] - c.campos[0];
    float dy = mf[1] - c.campos[1];
    float dz = mf[2] - c.campos[2];
    const float len = sqrtf(dx * dx + dy * dy + dz * dz);
    const float inv = 1.0f / len;
    dx *= inv;
    dy *= inv;
    dz *= inv;
    float Y[16];
    sh_basis(dx, dy, dz, deg, Y);
    float w[16];
#pragma unroll
    for (int j = 0; j < nb; ++j) {
      float s = 0.f;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        g_sh[j * 3 + ch] += Y[j] * grgb[ch];
        s += prm.sh[(size_t)(j * 3 + ch) * n + i] * grgb[ch];
      }
      w[j] = s;
    }
    float gx = 0.f, gy = 0.f, gz = 0.f;
    sh_basis_grad_dot(dx, dy, dz, deg, w, gx, gy, gz);
    const float dot = gx * dx + gy * dy + gz * dz;
    gmf[0] += (gx - dx * dot) * inv;
    gmf[1] += (gy - dy * dot) * inv;
    gmf[2] += (gz - dz * dot) * inv;
  }
  for (int k = 0; k < 3; ++k) g_mu[k] += (double)gmf[k];

  // ---- 3. scale and rotation from dL/dSigma3; opacity
  double g_ls[3] = {0, 0, 0}, g_q[4] = {0, 0, 0, 0}, g_logit = 0;
  if (loaded) {
    Body b;
    load_body(prm, i, b);
    const double G[9] = {Gs[0], Gs[1], Gs[2], Gs[1], Gs[3], Gs[4], Gs[2], Gs[4], Gs[5]};
    // Sigma3 = M M^T, M = Rq diag(s)
    double M[9];
    for (int r = 0; r < 3; ++r)
      for (int q = 0; q < 3; ++q) M[r * 3 + q] = b.Rq[r * 3 + q] * b.s[q];
    double gM[9];
    for (int r = 0; r < 3; ++r)
      for (int q = 0; q < 3; ++q)
        gM[r * 3 + q] = G[r * 3 + 0] * M[0 * 3 + q] + G[r * 3 + 1] * M[1 * 3 + q] +
                        G[r * 3 + 2] * M[2 * 3 + q];
    double gR[9];
    for (int r = 0; r < 3; ++r)
      for (int q = 0; q < 3; ++q) gR[r * 3 + q] = gM[r * 3 + q] * b.s[q];
    for (int q = 0; q < 3; ++q) {
      const double gsq = gM[0 * 3 + q] * b.Rq[0 * 3 + q] + gM[1 * 3 + q] * b.Rq[1 * 3 + q] +
                         gM[2 * 3 + q] * b.Rq[2 * 3 + q];
      g_ls[q] = gsq * b.s[q];
    }
    // rotation of the unit quaternion, entry by entry
    const double w = b.qn[0], x = b.qn[1], y = b.qn[2], z = b.qn[3];
    const double* g = gR;
    const double gw = 2 * (-z * g[1] + y * g[2] + z * g[3] - x * g[5] - y * g[6] + x * g[7]);
    const double gx = 2 * (y * g[1] + z * g[2] + y * g[3] - 2 * x * g[4] - w * g[5] + z * g[6] +
                           w * g[7] - 2 * x * g[8]);
    const double gy = 2 * (-2 * y * g[0] + x * g[1] + w * g[2] + x * g[3] + z * g[5] - w * g[6] +
                           z * g[7] - 2 * y * g[8]);
    const double gz = 2 * (-2 * z * g[0] - w * g[1] + x * g[2] + w * g[3] - 2 * z * g[4] +
                           y * g[5] + x * g[6] + y * g[7]);
    const double dot = w * gw + x * gx + y * gy + z * gz;
    g_q[0] = (gw - w * dot) / b.qnorm;
    g_q[1] = (gx - x * dot) / b.qnorm;
    g_q[2] = (gy - y * dot) / b.qnorm;
    g_q[3] = (gz - z * dot) / b.qnorm;
    const double op = 1.0 / (1.0 + exp(-(double)prm.logits[i]));
    g_logit = g_op * op * (1.0 - op);
  }
  // write (or add) the gradients; untouched Gaussians get zeros
  const bool add = gout.accumulate != 0;
  auto put = [&](float* dst, double val) {
    if (add) {
      if (any) *dst += (float)val;
    } else {
      *dst = (float)val;
    }
  };
  for (int k = 0; k < 3; ++k) put(gout.means + (size_t)k * n + i, g_mu[k]);
  for (int k = 0; k < 3; ++k) put(gout.log_scales + (size_t)k * n + i, g_ls[k]);
  for (int k = 0; k < 4; ++k) put(gout.quats + (size_t)k * n + i, g_q[k]);
  put(gout.logits + i, g_logit);
#pragma unroll
  for (int j = 0; j < nb * 3; ++j) put(gout.sh + (size_t)j * n + i, (double)g_sh[j]);
}

}  // namespace

gs_status launch_preprocess_fwd(const ParamsDev& p, const ViewTable& vt, Frame& f,
                                hipStream_t s) {
  const int blocks = (int)((p.n + 255) / 256);
  auto* sp = (float4*)f.splat.p;
  auto* rc = (uint2*)f.rect.p;
  auto* dk = (uint32_t*)f.dkey.p;
  auto* cm = (uint8_t*)f.clampm.p;
  switch (p.sh_degree) {
    case 0: hipLaunchKernelGGL(k_preprocess_fwd<0>, dim3(blocks), dim3(256), 0, s, p, vt, sp, rc, dk, cm); break;
    case 1: hipLaunchKernelGGL(k_preprocess_fwd<1>, dim3(blocks), dim3(256), 0, s, p, vt, sp, rc, dk, cm); break;
    case 2: hipLaunchKernelGGL(k_preprocess_fwd<2>, dim3(blocks), dim3(256), 0, s, p, vt, sp, rc, dk, cm); break;
    default: hipLaunchKernelGGL(k_preprocess_fwd<3>, dim3(blocks), dim3(256), 0, s, p, vt, sp, rc, dk, cm); break;
  }
  GS_LAUNCHED("preprocess_fwd");
  return GS_OK;
}

gs_status launch_preprocess_bwd(const ParamsDev& p, const ViewTable& vt, Frame& f,
                                const GradsDev& g, hipStream_t s) {
  const int blocks = (int)((p.n + 255) / 256);
  auto* ac = (float*)f.acc.p;
  auto* rc = (const uint2*)f.rect.p;
  auto* cm = (const uint8_t*)f.clampm.p;
  switch (p.sh_degree) {
    case 0: hipLaunchKernelGGL(k_preprocess_bwd<0>, dim3(blocks), dim3(256), 0, s, p, vt, ac, rc, cm, g); break;
    case 1: hipLaunchKernelGGL(k_preprocess_bwd<1>, dim3(blocks), dim3(256), 0, s, p, vt, ac, rc, cm, g); break;
    case 2: hipLaunchKernelGGL(k_preprocess_bwd<2>, dim3(blocks), dim3(256), 0, s, p, vt, ac, rc, cm, g); break;
    default: hipLaunchKernelGGL(k_preprocess_bwd<3>, dim3(blocks), dim3(256), 0, s, p, vt, ac, rc, cm, g); break;
  }
  GS_LAUNCHED("preprocess_bwd");
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

__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n1 = (uint32_t)p1;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    const uint32_t n3 = (uint32_t)p0;
    c[0] = n0;
    c[1] = n1;
    c[2] = n2;
    c[3] = n3;
  }
}

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
