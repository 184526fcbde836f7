// Per-surfel preprocessing: sort key, cull, screen tile rectangle and the
// FP32 record the collection pass evaluates per pixel; and its backward.
//
// Paper: surfels are preprocessed and sorted by the depth of their centres
// before tile-based compositing (Preliminaries, 2D Gaussian Splatting); the
// ray-surfel intersection (u, v, t*) follows 2DGS (Representation, Geometry
// and Appearance).
//
// The binning arithmetic runs in FP64 with contraction disabled and a fixed
// evaluation order (dot products left to right, one rounding per operation),
// so the depth keys and tile rectangles are exact functions of the inputs.
//
// The record re-expresses the ray-plane intersection per pixel offset
// (dx, dy) from the projected centre m: with c = mu_cam / mu_cam.z,
// n the camera-frame normal, k = c.n, a_i = R_cw v_i / s_i and
// B_i = a_i - n (c.a_i) / k,
//   den = 1 + dx n_x/(k fx) + dy n_y/(k fy),   t = mu_cam.z / den,
//   u   = mu_cam.z (dx B1_x/fx + dy B1_y/fy) / den  (v likewise with B2).
// Only pixel offsets enter the FP32 per-pixel arithmetic, so it does not
// lose digits to the absolute pixel position or the depth.
#include <math.h>

#include "nx_internal.h"

namespace nx {
namespace {

__device__ __forceinline__ bool finite_f(float x) { return isfinite(x); }

// Columns of the unit-quaternion rotation matrix, q = (w, x, y, z).
__device__ void quat_cols_exact(double w, double x, double y, double z, double v1[3], double v2[3],
                                double v3[3]) {
#pragma clang fp contract(off)
  v1[0] = 1.0 - 2.0 * ((y * y) + (z * z));
  v1[1] = 2.0 * ((x * y) + (w * z));
  v1[2] = 2.0 * ((x * z) - (w * y));
  v2[0] = 2.0 * ((x * y) - (w * z));
  v2[1] = 1.0 - 2.0 * ((x * x) + (z * z));
  v2[2] = 2.0 * ((y * z) + (w * x));
  v3[0] = 2.0 * ((x * z) + (w * y));
  v3[1] = 2.0 * ((y * z) - (w * x));
  v3[2] = 1.0 - 2.0 * ((x * x) + (y * y));
}

__device__ void to_cam_exact(const CamDev& c, const double p[3], double o[3]) {
#pragma clang fp contract(off)
  for (int k = 0; k < 3; ++k)
    o[k] = (((c.m[4 * k] * p[0]) + (c.m[4 * k + 1] * p[1])) + (c.m[4 * k + 2] * p[2])) + c.m[4 * k + 3];
}

// Tile rectangle of the support quad clipped to z > near. Returns the number
// of covered tiles (0 if none) and writes tx0, ty0, tx1, ty1.
__device__ int tile_rect_exact(const CamDev& c, const double mu[3], const double v1[3], const double v2[3],
                               double s1, double s2, int4* rect) {
#pragma clang fp contract(off)
  const double r1 = 3.0 * s1;
  const double r2 = 3.0 * s2;
  const double sa[4] = {-1.0, 1.0, 1.0, -1.0};
  const double sb[4] = {-1.0, -1.0, 1.0, 1.0};
  double cc[4][3];
  for (int i = 0; i < 4; ++i) {
    const double ra = sa[i] * r1;
    const double rb = sb[i] * r2;
    double p[3];
    for (int k = 0; k < 3; ++k) p[k] = (mu[k] + (ra * v1[k])) + (rb * v2[k]);
    to_cam_exact(c, p, cc[i]);
  }
  double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
  int nv = 0;
  for (int i = 0; i < 4; ++i) {
    const double* A = cc[i];
    const double* B = cc[(i + 1) & 3];
    const bool ina = A[2] > c.near_z;
    const bool inb = B[2] > c.near_z;
    double V[2][3];
    int nout = 0;
    if (ina) {
      V[nout][0] = A[0];
      V[nout][1] = A[1];
      V[nout][2] = A[2];
      ++nout;
    }
    if (ina != inb) {
      const double s = (c.near_z - A[2]) / (B[2] - A[2]);
      for (int k = 0; k < 3; ++k) V[nout][k] = A[k] + (s * (B[k] - A[k]));
      ++nout;
    }
    for (int j = 0; j < nout; ++j) {
      const double X = (c.fx * (V[j][0] / V[j][2])) + c.cx;
      const double Y = (c.fy * (V[j][1] / V[j][2])) + c.cy;
      xmin = fmin(xmin, X);
      xmax = fmax(xmax, X);
      ymin = fmin(ymin, Y);
      ymax = fmax(ymax, Y);
      ++nv;
    }
  }
  if (nv == 0) return -1;
  const double ftx0 = floor((xmin - kMarginPx) / (double)kTile);
  const double ftx1 = floor((xmax + kMarginPx) / (double)kTile);
  const double fty0 = floor((ymin - kMarginPx) / (double)kTile);
  const double fty1 = floor((ymax + kMarginPx) / (double)kTile);
  const int tx0 = (int)fmin(fmax(ftx0, 0.0), (double)c.ntx);
  const int tx1 = (int)fmin(fmax(ftx1, -1.0), (double)(c.ntx - 1));
  const int ty0 = (int)fmin(fmax(fty0, 0.0), (double)c.nty);
  const int ty1 = (int)fmin(fmax(fty1, -1.0), (double)(c.nty - 1));
  *rect = make_int4(tx0, ty0, tx1, ty1);
  if (tx0 > tx1 || ty0 > ty1) return 0;
  return (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
}

// Scalar type with one forward-mode derivative, for the record Jacobian.
struct Dual {
  double v, d;
  __device__ Dual() : v(0), d(0) {}
  __device__ Dual(double a) : v(a), d(0) {}
  __device__ Dual(double a, double b) : v(a), d(b) {}
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
  const double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
__device__ __forceinline__ double val(double a) { return a; }
__device__ __forceinline__ double val(Dual a) { return a.v; }

__device__ __forceinline__ Dual sqrt_d(Dual a) {
  const double r = sqrt(a.v);
  return Dual(r, a.d / (2.0 * r));
}
__device__ __forceinline__ double sqrt_d(double a) { return sqrt(a); }

// Real spherical harmonics up to degree 3 of a unit direction (x, y, z), in
// the usual Cartesian form with orthonormal constants (Representation,
// Appearance: channel-wise coefficients, 16 per channel). The colour of a
// channel is sum_k Y_k a_k + 0.5, clamped below at 0.
template <typename T>
__device__ void sh_basis16(T x, T y, T z, T Y[16]) {
  const double C0 = 0.28209479177387814, C1 = 0.4886025119029199;
  const double C2[5] = {1.0925484305920792, -1.0925484305920792, 0.31539156525252005, -1.0925484305920792,
                        0.5462742152960396};
  const double C3[7] = {-0.5900435899266435, 2.890611442640554, -0.4570457994644658, 0.3731763325901154,
                        -0.4570457994644658, 1.445305721320277, -0.5900435899266435};
  const T xx = x * x, yy = y * y, zz = z * z;
  Y[0] = T(C0);
  Y[1] = T(-C1) * y;
  Y[2] = T(C1) * z;
  Y[3] = T(-C1) * x;
  Y[4] = T(C2[0]) * (x * y);
  Y[5] = T(C2[1]) * (y * z);
  Y[6] = T(C2[2]) * (T(2.0) * zz - xx - yy);
  Y[7] = T(C2[3]) * (x * z);
  Y[8] = T(C2[4]) * (xx - yy);
  Y[9] = T(C3[0]) * y * (T(3.0) * xx - yy);
  Y[10] = T(C3[1]) * (x * y) * z;
  Y[11] = T(C3[2]) * y * (T(4.0) * zz - xx - yy);
  Y[12] = T(C3[3]) * z * (T(2.0) * zz - T(3.0) * xx - T(3.0) * yy);
  Y[13] = T(C3[4]) * x * (T(4.0) * zz - xx - yy);
  Y[14] = T(C3[5]) * z * (xx - yy);
  Y[15] = T(C3[6]) * x * (xx - T(3.0) * yy);
}

// The three channels before the clamp, sum_k Y_k(d) a_{3k+c} + 0.5, for the
// unit direction d from the camera centre o to the surfel centre mu.
template <typename T>
__device__ void sh_colour_raw(const T mu[3], const double o[3], const float* a, T rgb[3]) {
  const T dx = mu[0] - T(o[0]), dy = mu[1] - T(o[1]), dz = mu[2] - T(o[2]);
  const T len = sqrt_d(dx * dx + dy * dy + dz * dz);
  T Y[16];
  sh_basis16<T>(dx / len, dy / len, dz / len, Y);
  for (int c = 0; c < 3; ++c) {
    T acc(0.5);
    for (int k = 0; k < 16; ++k) acc = acc + Y[k] * T((double)a[3 * k + c]);
    rgb[c] = acc;
  }
}

// World-space camera centre o = -R^T t.
__device__ __forceinline__ void camera_centre(const CamDev& c, double o[3]) {
  for (int k = 0; k < 3; ++k) o[k] = -(c.m[k] * c.m[3] + c.m[4 + k] * c.m[7] + c.m[8 + k] * c.m[11]);
}

template <typename T>
struct Geo {
  T mx, my, p1x, p1y, p2x, p2y, qx, qy, mz;
  bool degenerate;
};

// Record geometry (m, P1, P2, Q, mz) from mu, q, s for one camera.
template <typename T>
__device__ Geo<T> record_geometry(const CamDev& c, const T mu[3], const T q[4], const T s[2]) {
  const T w = q[0], x = q[1], y = q[2], z = q[3];
  const T one(1.0), two(2.0);
  T v1[3] = {one - two * (y * y + z * z), two * (x * y + w * z), two * (x * z - w * y)};
  T v2[3] = {two * (x * y - w * z), one - two * (x * x + z * z), two * (y * z + w * x)};
  T v3[3] = {two * (x * z + w * y), two * (y * z - w * x), one - two * (x * x + y * y)};
  T muc[3], n[3], e1[3], e2[3];
  for (int k = 0; k < 3; ++k) {
    const T r0(c.m[4 * k]), r1(c.m[4 * k + 1]), r2(c.m[4 * k + 2]);
    muc[k] = r0 * mu[0] + r1 * mu[1] + r2 * mu[2] + T(c.m[4 * k + 3]);
    n[k] = r0 * v3[0] + r1 * v3[1] + r2 * v3[2];
    e1[k] = r0 * v1[0] + r1 * v1[1] + r2 * v1[2];
    e2[k] = r0 * v2[0] + r1 * v2[1] + r2 * v2[2];
  }
  Geo<T> g;
  g.mz = muc[2];
  const T cx = muc[0] / muc[2], cy = muc[1] / muc[2];
  const T fx(c.fx), fy(c.fy);
  g.mx = fx * cx + T(c.cx);
  g.my = fy * cy + T(c.cy);
  const T k = cx * n[0] + cy * n[1] + n[2];
  g.degenerate = !(val(k) != 0.0);
  if (g.degenerate) return g;
  T a1[3], a2[3];
  for (int i = 0; i < 3; ++i) {
    a1[i] = e1[i] / s[0];
    a2[i] = e2[i] / s[1];
  }
  const T ca1 = (cx * a1[0] + cy * a1[1] + a1[2]) / k;
  const T ca2 = (cx * a2[0] + cy * a2[1] + a2[2]) / k;
  const T b1x = a1[0] - n[0] * ca1, b1y = a1[1] - n[1] * ca1;
  const T b2x = a2[0] - n[0] * ca2, b2y = a2[1] - n[1] * ca2;
  g.p1x = g.mz * b1x / fx;
  g.p1y = g.mz * b1y / fy;
  g.p2x = g.mz * b2x / fx;
  g.p2y = g.mz * b2y / fy;
  g.qx = n[0] / (k * fx);
  g.qy = n[1] / (k * fy);
  return g;
}

__global__ __launch_bounds__(256) void preprocess_kernel(const float* __restrict__ means,
                                                         const float* __restrict__ quats,
                                                         const float* __restrict__ scales,
                                                         const float* __restrict__ opac,
                                                         const float* __restrict__ gammas,
                                                         const float* __restrict__ colors, int sh, int64_t n,
                                                         CamDev cam, uint32_t* __restrict__ depth_keys,
                                                         uint32_t* __restrict__ tile_counts,
                                                         int4* __restrict__ rects, float4* __restrict__ records) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float fm[3] = {means[3 * i], means[3 * i + 1], means[3 * i + 2]};
  const float fq[4] = {quats[4 * i], quats[4 * i + 1], quats[4 * i + 2], quats[4 * i + 3]};
  const float fs[2] = {scales[2 * i], scales[2 * i + 1]};
  const float fo = opac[i];
  const float fg[2] = {gammas[2 * i], gammas[2 * i + 1]};
  const int nc = sh ? 48 : 3;  // colour values per surfel: RGB, or 16 SH coefficients per channel
  const float* col = colors + (int64_t)nc * i;
  bool ok = true;
  for (int k = 0; k < nc; ++k) ok &= finite_f(col[k]);
  for (int k = 0; k < 3; ++k) ok &= finite_f(fm[k]);
  for (int k = 0; k < 4; ++k) ok &= finite_f(fq[k]);
  for (int k = 0; k < 2; ++k) ok &= finite_f(fs[k]) && finite_f(fg[k]);
  ok &= finite_f(fo);
  ok &= (fs[0] > 0.0f) && (fs[1] > 0.0f);

  double mu[3] = {fm[0], fm[1], fm[2]};
  double v1[3], v2[3], v3[3];
  quat_cols_exact(fq[0], fq[1], fq[2], fq[3], v1, v2, v3);
  double muc[3];
  to_cam_exact(cam, mu, muc);
  const float key = (float)muc[2];
  ok &= muc[2] > cam.near_z;

  int count = 0;
  int4 rect = make_int4(0, 0, -1, -1);
  if (ok) {
    const int r = tile_rect_exact(cam, mu, v1, v2, (double)fs[0], (double)fs[1], &rect);
    if (r < 0) ok = false;
    count = r > 0 ? r : 0;
  }
  depth_keys[i] = ok ? __float_as_uint(key) : 0xFFFFFFFFu;
  tile_counts[i] = ok ? (uint32_t)count : 0u;
  rects[i] = rect;

  float4 rec[kRecF4];
  for (int k = 0; k < kRecF4; ++k) rec[k] = make_float4(0.f, 0.f, 0.f, 0.f);
  if (ok && count > 0) {
    const double dq[4] = {fq[0], fq[1], fq[2], fq[3]};
    const double ds[2] = {fs[0], fs[1]};
    const Geo<double> g = record_geometry<double>(cam, mu, dq, ds);
    float fc[3] = {col[0], col[1], col[2]};
    if (sh) {
      double o[3], rgb[3];
      camera_centre(cam, o);
      sh_colour_raw<double>(mu, o, col, rgb);
      for (int c = 0; c < 3; ++c) fc[c] = (float)fmax(rgb[c], 0.0);
    }
    if (!g.degenerate) {
      const double mxi = floor(g.mx), myi = floor(g.my);
      rec[0] = make_float4((float)mxi, (float)myi, (float)(0.5 - (g.mx - mxi)), (float)(0.5 - (g.my - myi)));
      rec[1] = make_float4((float)g.p1x, (float)g.p1y, (float)g.p2x, (float)g.p2y);
      rec[2] = make_float4((float)g.qx, (float)g.qy, (float)g.mz, fo);
      rec[3] = make_float4(fg[0], fg[1], fc[0], fc[1]);
      rec[4] = make_float4(fc[2], 0.f, 0.f, 0.f);
    }
    // A degenerate plane (through the camera centre) keeps opacity 0 and is never composited.
  }
  for (int k = 0; k < kRecF4; ++k) records[(int64_t)kRecF4 * i + k] = rec[k];
}

__global__ __launch_bounds__(256) void preprocess_backward_kernel(
    const float* __restrict__ means, const float* __restrict__ quats, const float* __restrict__ scales, int64_t n,
    const float* __restrict__ colors, int sh, CamDev cam, const uint32_t* __restrict__ tile_counts,
    const float* __restrict__ rg, float* g_means, float* g_quats, float* g_scales, float* g_opac, float* g_gammas,
    float* g_colors, float* g_blended) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (tile_counts[i] == 0) return;
  const float* r = rg + (int64_t)kRecGrad * i;
  if (g_blended && r[15] != 0.0f) g_blended[i] += r[15];
  float gr[15];
  bool any = false;
  for (int k = 0; k < 15; ++k) {
    gr[k] = r[k];
    any |= gr[k] != 0.0f;
  }
  if (!any) return;
  if (g_opac) g_opac[i] += gr[9];
  if (g_gammas) {
    g_gammas[2 * i] += gr[10];
    g_gammas[2 * i + 1] += gr[11];
  }
  double sh_mu[3] = {0.0, 0.0, 0.0};  // gradient reaching mu through the view direction
  if (sh) {
    // c = max(0, sum_k Y_k(d) a_k + 0.5), d = (mu - o) / |mu - o|:
    // dL/da_{3k+c} = [raw_c > 0] Y_k dL/dc, and dL/dmu by forward mode in mu.
    const float* a = colors + (int64_t)48 * i;
    double o[3];
    camera_centre(cam, o);
    const double m0[3] = {means[3 * i], means[3 * i + 1], means[3 * i + 2]};
    double rgb[3];
    sh_colour_raw<double>(m0, o, a, rgb);
    double gc[3];
    for (int c = 0; c < 3; ++c) gc[c] = rgb[c] > 0.0 ? (double)gr[12 + c] : 0.0;
    if (g_colors) {
      const double dx = m0[0] - o[0], dy = m0[1] - o[1], dz = m0[2] - o[2];
      const double len = sqrt(dx * dx + dy * dy + dz * dz);
      double Y[16];
      sh_basis16<double>(dx / len, dy / len, dz / len, Y);
      for (int k = 0; k < 16; ++k)
        for (int c = 0; c < 3; ++c)
          if (gc[c] != 0.0) g_colors[48 * i + 3 * k + c] += (float)(Y[k] * gc[c]);
    }
    for (int j = 0; j < 3; ++j) {
      Dual m[3];
      for (int k = 0; k < 3; ++k) m[k] = Dual(m0[k], k == j ? 1.0 : 0.0);
      Dual c3[3];
      sh_colour_raw<Dual>(m, o, a, c3);
      sh_mu[j] = gc[0] * c3[0].d + gc[1] * c3[1].d + gc[2] * c3[2].d;
    }
  } else if (g_colors) {
    g_colors[3 * i] += gr[12];
    g_colors[3 * i + 1] += gr[13];
    g_colors[3 * i + 2] += gr[14];
  }
  // Vector-Jacobian product of the record geometry, one forward-mode pass
  // per input (mu: 3, q: 4, s: 2).
  const double base[9] = {means[3 * i],     means[3 * i + 1], means[3 * i + 2], quats[4 * i],
                          quats[4 * i + 1], quats[4 * i + 2], quats[4 * i + 3], scales[2 * i],
                          scales[2 * i + 1]};
  double out[9];
  for (int dir = 0; dir < 9; ++dir) {
    Dual in[9];
    for (int k = 0; k < 9; ++k) in[k] = Dual(base[k], k == dir ? 1.0 : 0.0);
    const Geo<Dual> g = record_geometry<Dual>(cam, in, in + 3, in + 7);
    if (g.degenerate) return;
    out[dir] = gr[0] * g.mx.d + gr[1] * g.my.d + gr[2] * g.p1x.d + gr[3] * g.p1y.d + gr[4] * g.p2x.d +
               gr[5] * g.p2y.d + gr[6] * g.qx.d + gr[7] * g.qy.d + gr[8] * g.mz.d;
  }
  for (int k = 0; k < 3; ++k) out[k] += sh_mu[k];
  if (g_means)
    for (int k = 0; k < 3; ++k) g_means[3 * i + k] += (float)out[k];
  if (g_quats)
    for (int k = 0; k < 4; ++k) g_quats[4 * i + k] += (float)out[3 + k];
  if (g_scales)
    for (int k = 0; k < 2; ++k) g_scales[2 * i + k] += (float)out[7 + k];
}

}  // namespace

hipError_t launch_preprocess(const float* means, const float* quats, const float* scales, const float* opac,
                             const float* gammas, const float* colors, int sh, int64_t n, const CamDev& cam,
                             uint32_t* depth_keys, uint32_t* tile_counts, int4* rects, float4* records,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(preprocess_kernel, dim3((unsigned)blocks), dim3(256), 0, s, means, quats, scales, opac, gammas,
                     colors, sh, n, cam, depth_keys, tile_counts, rects, records);
  return hipGetLastError();
}

hipError_t launch_preprocess_backward(const float* means, const float* quats, const float* scales,
                                      const float* colors, int sh, int64_t n, const CamDev& cam,
                                      const uint32_t* tile_counts, const float* rec_grad, float* g_means,
                                      float* g_quats, float* g_scales, float* g_opac, float* g_gammas,
                                      float* g_colors, float* g_blended, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(preprocess_backward_kernel, dim3((unsigned)blocks), dim3(256), 0, s, means, quats, scales, n,
                     colors, sh, cam, tile_counts, rec_grad, g_means, g_quats, g_scales, g_opac, g_gammas, g_colors,
                     g_blended);
  return hipGetLastError();
}

}  // namespace nx
