// Collection pass (forward) and its replay (backward), one 16x16 tile per
// 256-thread workgroup, one pixel per thread.
//
// Paper, Rendering, Collection Pass: per pixel the surfels are composited
// front to back (eq. composite); the blending weights w = alpha T select,
// through a K-entry buffer of (id, weight, depth), the K intersections of
// highest weight; N (eq. notexture) is the plain-colour render without them.
// Kernel: generalised Gaussian alpha = o exp(-|u|^{2 g1}/2) exp(-|v|^{2 g2}/2)
// (Representation, Geometry).
//
// Per tile the sorted surfel list is staged through LDS 256 records at a time
// (one record load per thread, then every thread reads each record as a
// broadcast). The workgroup leaves the list as soon as every pixel is done.
//
// The backward replays each pixel front to back, recomputing alpha and T with
// the same instructions as the forward, so every decision is reproduced
// exactly. With S_i = sum_{k>i} w_k dL/dw_k it uses
//   dL/dalpha_i = T_i dL/dw_i - S_i / (1 - alpha_i),
// where S starts at sum_k w_k dL/dw_k = g.N + sum_j W_j (g.Tex_j + dL/dW_j)
// (all forward outputs) and drops by w_i dL/dw_i at every step. Per surfel
// the 15 record gradients, and with a per-pixel error map the blended error
// w_i E_p, are reduced across the wavefront and added with one atomic per
// value.
#include <math.h>

#include "nx_internal.h"

namespace nx {
namespace {

// Records staged in LDS per batch: B of them, one per thread of the first B
// (B in {64, 128, 256}; chosen per context, see launch_raster_forward).
constexpr float kNegHalfLog2e = -0.72134752044448170368f;
constexpr float kLn2 = 0.69314718055994530942f;

struct PairEval {
  float dx, dy, inv, t, u, v, pu, pv, G, araw, alpha;
};

__device__ __forceinline__ float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float log2_fast(float x) { return __builtin_amdgcn_logf(x); }

// |a|^e for e >= 1 (0 at a = 0).
__device__ __forceinline__ float abs_pow(float a, float e) {
  const float aa = fabsf(a);
  return aa > 0.0f ? exp2_fast(e * log2_fast(aa)) : 0.0f;
}

// Ray-surfel intersection and alpha of one (pixel, record) pair. Returns
// true if the pair is composited candidate (inside the support, in front of
// the near plane, alpha >= 1/255). Shared verbatim by forward and backward.
__device__ __forceinline__ bool eval_pair(const float4& r0, const float4& r1, const float4& r2, const float4& r3,
                                          float pxf, float pyf, float near_z, PairEval& e) {
  e.dx = (pxf - r0.x) + r0.z;
  e.dy = (pyf - r0.y) + r0.w;
  const float den = fmaf(e.dx, r2.x, fmaf(e.dy, r2.y, 1.0f));
  e.inv = __builtin_amdgcn_rcpf(den);
  e.t = r2.z * e.inv;
  e.u = fmaf(e.dx, r1.x, e.dy * r1.y) * e.inv;
  e.v = fmaf(e.dx, r1.z, e.dy * r1.w) * e.inv;
  // one combined test (bitwise, not short-circuit: each && would become a
  // branch on the execution mask)
  if (!((e.t > near_z) & (fabsf(e.u) <= kSupport) & (fabsf(e.v) <= kSupport))) return false;
  if (r3.x == 1.0f && r3.y == 1.0f) {
    e.pu = e.u * e.u;
    e.pv = e.v * e.v;
  } else {
    e.pu = abs_pow(e.u, 2.0f * r3.x);
    e.pv = abs_pow(e.v, 2.0f * r3.y);
  }
  e.G = exp2_fast(kNegHalfLog2e * (e.pu + e.pv));
  e.araw = r2.w * e.G;
  e.alpha = fminf(e.araw, kAlphaMax);
  return e.alpha >= kAlphaMin;
}

struct TileCoords {
  int px, py;
  bool inside;
};

__device__ __forceinline__ TileCoords tile_pixel(int tile, int ntx, int width, int height) {
  const int tx = tile % ntx, ty = tile / ntx;
  TileCoords c;
  c.px = tx * kTile + (threadIdx.x & (kTile - 1));
  c.py = ty * kTile + (threadIdx.x >> 4);
  c.inside = c.px < width && c.py < height;
  return c;
}

template <int K, int B>
__global__ __launch_bounds__(256) void raster_forward_kernel(const float4* __restrict__ records,
                                                             const uint32_t* __restrict__ sorted_ids,
                                                             const uint2* __restrict__ ranges, int ntx, int width,
                                                             int height, float near_z, float* __restrict__ plain,
                                                             int32_t* __restrict__ out_ids,
                                                             float* __restrict__ out_w, float* __restrict__ out_d,
                                                             float* __restrict__ t_final,
                                                             uint32_t* __restrict__ n_iter) {
  __shared__ float4 s_rec[B * kRecF4];
  __shared__ uint32_t s_id[B];
  const int tile = blockIdx.x;
  const TileCoords pc = tile_pixel(tile, ntx, width, height);
  const uint2 range = ranges[tile];
  const float pxf = (float)pc.px, pyf = (float)pc.py;

  float T = 1.0f, cr = 0.0f, cg = 0.0f, cb = 0.0f;
  constexpr int KB = K > 0 ? K : 1;
  float kw[KB], kd[KB];
  int kid[KB];
#pragma unroll
  for (int s = 0; s < KB; ++s) {
    kw[s] = 0.0f;
    kd[s] = 0.0f;
    kid[s] = -1;
  }
  int kn = 0;
  uint32_t last = 0;
  bool done = !pc.inside;

  for (uint32_t start = range.x; start < range.y; start += B) {
    if (__syncthreads_and(done)) break;
    const uint32_t idx = start + threadIdx.x;
    if (threadIdx.x < B && idx < range.y) {
      const uint32_t id = sorted_ids[idx];
      s_id[threadIdx.x] = id;
#pragma unroll
      for (int f = 0; f < kRecF4; ++f) s_rec[threadIdx.x * kRecF4 + f] = records[(int64_t)id * kRecF4 + f];
    }
    __syncthreads();
    const int cnt = (int)min((uint32_t)B, range.y - start);
    for (int j = 0; j < cnt; ++j) {
      if (done) continue;
      const float4 r0 = s_rec[j * kRecF4 + 0], r1 = s_rec[j * kRecF4 + 1], r2 = s_rec[j * kRecF4 + 2],
                   r3 = s_rec[j * kRecF4 + 3];
      PairEval e;
      if (!eval_pair(r0, r1, r2, r3, pxf, pyf, near_z, e)) continue;
      const float test_T = T * (1.0f - e.alpha);
      if (test_T < kTMin) {
        done = true;
        continue;
      }
      const float w = e.alpha * T;
      const float r4x = s_rec[j * kRecF4 + 4].x;
      cr = fmaf(w, r3.z, cr);
      cg = fmaf(w, r3.w, cg);
      cb = fmaf(w, r4x, cb);
      if (K > 0) {
        const int id = (int)s_id[j];
        if (kn < K) {
#pragma unroll
          for (int s = 0; s < KB; ++s)
            if (s == kn) {
              kw[s] = w;
              kid[s] = id;
              kd[s] = e.t;
            }
          ++kn;
        } else {
          // Worst entry under (weight desc, id asc); replace it if the new one is better.
          float ww = kw[0];
          int wi = kid[0], ws = 0;
#pragma unroll
          for (int s = 1; s < KB; ++s) {
            const bool worse = (kw[s] < ww) | ((kw[s] == ww) & (kid[s] > wi));
            ww = worse ? kw[s] : ww;
            wi = worse ? kid[s] : wi;
            ws = worse ? s : ws;
          }
          if ((w > ww) | ((w == ww) & (id < wi))) {
#pragma unroll
            for (int s = 0; s < KB - 1; ++s)
              if (s >= ws) {
                kw[s] = kw[s + 1];
                kid[s] = kid[s + 1];
                kd[s] = kd[s + 1];
              }
            kw[KB - 1] = w;
            kid[KB - 1] = id;
            kd[KB - 1] = e.t;
          }
        }
      }
      T = test_T;
      last = start - range.x + (uint32_t)j + 1u;
    }
  }
  if (!pc.inside) return;
  const int64_t p = (int64_t)pc.py * width + pc.px;
  // Remove the selected surfels' plain colours (eq. notexture).
#pragma unroll
  for (int s = 0; s < KB; ++s) {
    if (K > 0 && kid[s] >= 0) {
      const float4 a = records[(int64_t)kid[s] * kRecF4 + 3];
      const float b = records[(int64_t)kid[s] * kRecF4 + 4].x;
      cr = fmaf(-kw[s], a.z, cr);
      cg = fmaf(-kw[s], a.w, cg);
      cb = fmaf(-kw[s], b, cb);
    }
  }
  plain[3 * p] = cr;
  plain[3 * p + 1] = cg;
  plain[3 * p + 2] = cb;
  if (K > 0) {
#pragma unroll
    for (int s = 0; s < KB; ++s) {
      out_ids[p * K + s] = kid[s];
      out_w[p * K + s] = kw[s];
      out_d[p * K + s] = kd[s];
    }
  }
  t_final[p] = T;
  n_iter[p] = last;
}

// Sum of v[0..15] over the wavefront: each halving step keeps half of the
// values. Lane l ends with the total of value 8*b5 + 4*b4 + 2*b3 + b2
// (b = bits of l); lanes with l % 4 == 0 hold them. The exchanges across
// 32- and 16-lane halves are register swaps between two values (gfx950's
// permlane swaps: the upper half of the first value trades places with the
// lower half of the second), so each step is one swap and one add per pair;
// the steps within 16 lanes use DPP and the swizzle unit, no LDS permute.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
__device__ __forceinline__ float wave_transpose_sum16(float v[16], int lane, int* which) {
  float a8[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    // lanes 0-31 end with v[i] of lanes l and l + 32, lanes 32-63 with v[i + 8]
    const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 8]), false, false);
    a8[i] = __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
  }
  float a4[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    // even rows of 16 lanes end with a8[i] of rows r and r + 1, odd rows with a8[i + 4]
    const auto sw = __builtin_amdgcn_permlane16_swap(__float_as_uint(a8[i]), __float_as_uint(a8[i + 4]), false, false);
    a4[i] = __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
  }
  float a2[2];
  const bool h8 = lane & 8;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const float send = h8 ? a4[i] : a4[i + 2];
    const float keep = h8 ? a4[i + 2] : a4[i];
    a2[i] = keep + dpp_mov<0x128>(send);  // row_ror:8 = lane ^ 8
  }
  const bool h4 = lane & 4;
  const float send = h4 ? a2[0] : a2[1];
  float x = (h4 ? a2[1] : a2[0]) +
            __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(send), (4 << 10) | 0x1F));  // lane ^ 4
  x += dpp_mov<0x4E>(x);  // quad_perm [2,3,0,1] = lane ^ 2
  x += dpp_mov<0xB1>(x);  // quad_perm [1,0,3,2] = lane ^ 1
  *which = ((lane & 32) ? 8 : 0) + ((lane & 16) ? 4 : 0) + (h8 ? 2 : 0) + (h4 ? 1 : 0);
  return x;
}

template <int K, int B>
__global__ __launch_bounds__(256) void raster_backward_kernel(
    const float4* __restrict__ records, const uint32_t* __restrict__ sorted_ids, const uint2* __restrict__ ranges,
    int ntx, int width, int height, float near_z, const float* __restrict__ plain, const int32_t* __restrict__ ids,
    const float* __restrict__ weights, const float* __restrict__ tex, const uint32_t* __restrict__ n_iter,
    const float* __restrict__ grad_image, const float* __restrict__ grad_weights,
    const float* __restrict__ grad_depth, const float* __restrict__ pixel_error, float* __restrict__ rec_grad) {
  __shared__ float4 s_rec[B * kRecF4];
  __shared__ uint32_t s_id[B];
  const int tile = blockIdx.x;
  const TileCoords pc = tile_pixel(tile, ntx, width, height);
  const uint2 range = ranges[tile];
  const float pxf = (float)pc.px, pyf = (float)pc.py;
  const int lane = threadIdx.x & 63;

  constexpr int KB = K > 0 ? K : 1;
  float g0 = 0.f, g1 = 0.f, g2 = 0.f, S = 0.f, perr = 0.f;
  int kid[KB];
  float gsel[KB], gdep[KB];
  uint32_t my_n = 0;
#pragma unroll
  for (int s = 0; s < KB; ++s) {
    kid[s] = -1;
    gsel[s] = 0.f;
    gdep[s] = 0.f;
  }
  if (pc.inside) {
    const int64_t p = (int64_t)pc.py * width + pc.px;
    g0 = grad_image[3 * p];
    g1 = grad_image[3 * p + 1];
    g2 = grad_image[3 * p + 2];
    S = g0 * plain[3 * p] + g1 * plain[3 * p + 1] + g2 * plain[3 * p + 2];
    if (pixel_error) perr = pixel_error[p];
    if (K > 0) {
#pragma unroll
      for (int s = 0; s < KB; ++s) {
        kid[s] = ids[p * K + s];
        if (kid[s] >= 0) {
          const float* tx = tex + (p * K + s) * 3;
          float gs = g0 * tx[0] + g1 * tx[1] + g2 * tx[2];
          if (grad_weights) gs += grad_weights[p * K + s];
          gsel[s] = gs;
          gdep[s] = grad_depth ? grad_depth[p * K + s] : 0.f;
          S += weights[p * K + s] * gs;
        }
      }
    }
    my_n = n_iter[p];
  }
  float T = 1.0f;
  bool done = my_n == 0;

  for (uint32_t start = range.x; start < range.y; start += B) {
    if (__syncthreads_and(done)) break;
    const uint32_t idx = start + threadIdx.x;
    if (threadIdx.x < B && idx < range.y) {
      const uint32_t id = sorted_ids[idx];
      s_id[threadIdx.x] = id;
#pragma unroll
      for (int f = 0; f < kRecF4; ++f) s_rec[threadIdx.x * kRecF4 + f] = records[(int64_t)id * kRecF4 + f];
    }
    __syncthreads();
    const int cnt = (int)min((uint32_t)B, range.y - start);
    for (int j = 0; j < cnt; ++j) {
      const uint32_t rel = start - range.x + (uint32_t)j;
      if (rel >= my_n) done = true;
      const float4 r0 = s_rec[j * kRecF4 + 0], r1 = s_rec[j * kRecF4 + 1], r2 = s_rec[j * kRecF4 + 2],
                   r3 = s_rec[j * kRecF4 + 3];
      PairEval e;
      const bool active = !done && eval_pair(r0, r1, r2, r3, pxf, pyf, near_z, e);
      if (__ballot(active) == 0) continue;
      float gv[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) gv[k] = 0.0f;
      if (active) {
        const int id = (int)s_id[j];
        const float w = e.alpha * T;
        const float r4x = s_rec[j * kRecF4 + 4].x;
        bool sel = false;
        float Gi = 0.f, dLdt = 0.f;
#pragma unroll
        for (int s = 0; s < KB; ++s)
          if (K > 0 && kid[s] == id) {
            sel = true;
            Gi = gsel[s];
            dLdt = gdep[s];
          }
        if (!sel) {
          Gi = g0 * r3.z + g1 * r3.w + g2 * r4x;
          gv[12] = w * g0;
          gv[13] = w * g1;
          gv[14] = w * g2;
        }
        S -= w * Gi;
        const float one_m = 1.0f - e.alpha;
        // 1 - alpha >= 0.01 (alpha is clamped at 0.99): the hardware reciprocal
        // (1 ulp) instead of a correctly rounded division, a tenth of the
        // pair's instructions
        const float dLda = T * Gi - S * __builtin_amdgcn_rcpf(one_m);
        const float dLdraw = e.araw > kAlphaMax ? 0.0f : dLda;
        gv[9] = dLdraw * e.G;
        const float dLdE = -0.5f * e.G * r2.w * dLdraw;
        // E = |u|^(2 g1) + |v|^(2 g2): dE/du = 2 g1 |u|^(2 g1) / u, dE/dg1 = |u|^(2 g1) 2 ln|u|.
        const float au = fabsf(e.u), av = fabsf(e.v);
        float dLdu, dLdv;
        if (r3.x == 1.0f && r3.y == 1.0f) {
          dLdu = dLdE * 2.0f * e.u;
          dLdv = dLdE * 2.0f * e.v;
        } else {
          dLdu = au > 0.0f ? dLdE * e.pu * 2.0f * r3.x / e.u : 0.0f;
          dLdv = av > 0.0f ? dLdE * e.pv * 2.0f * r3.y / e.v : 0.0f;
        }
        gv[10] = au > 0.0f ? dLdE * e.pu * 2.0f * kLn2 * log2_fast(au) : 0.0f;
        gv[11] = av > 0.0f ? dLdE * e.pv * 2.0f * kLn2 * log2_fast(av) : 0.0f;
        const float dnu = dLdu * e.inv, dnv = dLdv * e.inv;
        const float dden = -(dLdu * e.u + dLdv * e.v + dLdt * e.t) * e.inv;
        gv[8] = dLdt * e.inv;
        gv[2] = dnu * e.dx;
        gv[3] = dnu * e.dy;
        gv[4] = dnv * e.dx;
        gv[5] = dnv * e.dy;
        gv[6] = dden * e.dx;
        gv[7] = dden * e.dy;
        gv[0] = -(dnu * r1.x + dnv * r1.z + dden * r2.x);
        gv[1] = -(dnu * r1.y + dnv * r1.w + dden * r2.y);
        gv[15] = w * perr;
        T *= one_m;
      }
      int which;
      const float tot = wave_transpose_sum16(gv, lane, &which);
      if ((lane & 3) == 0 && tot != 0.0f)
        atomicAdd(&rec_grad[(int64_t)s_id[j] * kRecGrad + which], tot);
    }
  }
}

template <int K, int B>
hipError_t launch_fwd_k1(const float4* records, const uint32_t* sorted_ids, const uint2* ranges, const CamDev& cam,
                        float* plain, int32_t* ids, float* weights, float* depths, float* t_final, uint32_t* n_iter,
                        hipStream_t s) {
  const int n_tiles = cam.ntx * cam.nty;
  hipLaunchKernelGGL((raster_forward_kernel<K, B>), dim3(n_tiles), dim3(256), 0, s, records, sorted_ids, ranges, cam.ntx,
                     cam.width, cam.height, (float)cam.near_z, plain, ids, weights, depths, t_final, n_iter);
  return hipGetLastError();
}

template <int K, int B>
hipError_t launch_bwd_k1(const float4* records, const uint32_t* sorted_ids, const uint2* ranges, const CamDev& cam,
                        const float* plain, const int32_t* ids, const float* weights, const float* tex,
                        const uint32_t* n_iter, const float* grad_image, const float* grad_weights,
                        const float* grad_depth, const float* pixel_error, float* rec_grad, hipStream_t s) {
  const int n_tiles = cam.ntx * cam.nty;
  hipLaunchKernelGGL((raster_backward_kernel<K, B>), dim3(n_tiles), dim3(256), 0, s, records, sorted_ids, ranges,
                     cam.ntx, cam.width, cam.height, (float)cam.near_z, plain, ids, weights, tex, n_iter, grad_image,
                     grad_weights, grad_depth, pixel_error, rec_grad);
  return hipGetLastError();
}

template <int K>
hipError_t launch_fwd_k(const float4* records, const uint32_t* sorted_ids, const uint2* ranges, const CamDev& cam,
                        float* plain, int32_t* ids, float* weights, float* depths, float* t_final, uint32_t* n_iter,
                        int batch, hipStream_t s) {
#define NX_FWD(BB) \
  return launch_fwd_k1<K, BB>(records, sorted_ids, ranges, cam, plain, ids, weights, depths, t_final, n_iter, s)
  switch (batch) {
    case 64: NX_FWD(64);
    case 128: NX_FWD(128);
    case 256: NX_FWD(256);
    default: return hipErrorInvalidValue;
  }
#undef NX_FWD
}

template <int K>
hipError_t launch_bwd_k(const float4* records, const uint32_t* sorted_ids, const uint2* ranges, const CamDev& cam,
                        const float* plain, const int32_t* ids, const float* weights, const float* tex,
                        const uint32_t* n_iter, const float* grad_image, const float* grad_weights,
                        const float* grad_depth, const float* pixel_error, float* rec_grad, int batch,
                        hipStream_t s) {
#define NX_BWD1(BB)                                                                                             \
  return launch_bwd_k1<K, BB>(records, sorted_ids, ranges, cam, plain, ids, weights, tex, n_iter, grad_image, \
                              grad_weights, grad_depth, pixel_error, rec_grad, s)
  switch (batch) {
    case 64: NX_BWD1(64);
    case 128: NX_BWD1(128);
    case 256: NX_BWD1(256);
    default: return hipErrorInvalidValue;
  }
#undef NX_BWD1
}

}  // namespace

hipError_t launch_raster_forward(int K, const float4* records, const uint32_t* sorted_ids, const uint2* ranges,
                                 const CamDev& cam, float* plain, int32_t* ids, float* weights, float* depths,
                                 float* t_final, uint32_t* n_iter, int batch, hipStream_t s) {
#define NX_FWD(KK) \
  return launch_fwd_k<KK>(records, sorted_ids, ranges, cam, plain, ids, weights, depths, t_final, n_iter, batch, s)
  switch (K) {
    case 0: NX_FWD(0);
    case 1: NX_FWD(1);
    case 2: NX_FWD(2);
    case 4: NX_FWD(4);
    case 8: NX_FWD(8);
    case 16: NX_FWD(16);
    default: return hipErrorInvalidValue;
  }
#undef NX_FWD
}

hipError_t launch_raster_backward(int K, const float4* records, const uint32_t* sorted_ids, const uint2* ranges,
                                  const CamDev& cam, const float* plain, const int32_t* ids, const float* weights,
                                  const float* tex, const uint32_t* n_iter, const float* grad_image,
                                  const float* grad_weights, const float* grad_depth, const float* pixel_error,
                                  float* rec_grad, int batch, hipStream_t s) {
#define NX_BWD(KK)                                                                                             \
  return launch_bwd_k<KK>(records, sorted_ids, ranges, cam, plain, ids, weights, tex, n_iter, grad_image, \
                          grad_weights, grad_depth, pixel_error, rec_grad, batch, s)
  switch (K) {
    case 0: NX_BWD(0);
    case 1: NX_BWD(1);
    case 2: NX_BWD(2);
    case 4: NX_BWD(4);
    case 8: NX_BWD(8);
    case 16: NX_BWD(16);
    default: return hipErrorInvalidValue;
  }
#undef NX_BWD
}

}  // namespace nx
