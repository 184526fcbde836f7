// Auxiliary losses of the optimisation and their gradients.
//
// Paper, Optimization, Losses:
//   L_texture = 1/(3P) sum_p sum_c | GT_pc - r_pc |, r_pc = sum_j W_pj Tex_pjc / S_p, S_p = sum_j W_pj
//               (pixels with S_p = 0 have no texture estimate and add nothing)
//   L_alpha   = 1/P sum_p (1 - S_p)
//   L_opacity = 1/N sum_i o_i
//   L_grid    = sum_l s_l^-3 sum_i sum_f H_lif^2 (the printed term is linear in
//               H; read as a weight decay normalised by the level's cell
//               volume, which is what keeps the entries near zero mean)
// Gradients, scaled by the caller's lambdas, are added to the buffers the
// rendering backward takes (dL/dW and dL/dTex feed nx_render_backward's
// optional inputs), to the opacity gradient and to the FP32 table gradient.
// The four unweighted loss values are summed per workgroup and added to a
// device array with float atomics (summation order varies run to run).
#include <hip/hip_fp16.h>

#include "nx_internal.h"

namespace nx {
namespace {

constexpr int kAuxThreads = 256;

// Sum of v over the workgroup, added to *dst by one thread.
__device__ __forceinline__ void block_add(float v, float* dst) {
  __shared__ float part[kAuxThreads / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) part[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int w = 0; w < kAuxThreads / 64; ++w) s += part[w];
    if (s != 0.f) atomicAdd(dst, s);
  }
  __syncthreads();
}

__global__ void zero4_kernel(float* losses) {
  if (threadIdx.x < 4) losses[threadIdx.x] = 0.f;
}

// One thread per pixel: L_alpha and L_texture terms and their gradients.
__global__ __launch_bounds__(kAuxThreads) void aux_pixel_kernel(int64_t P, int K, const float* __restrict__ W,
                                                                const float* __restrict__ tex,
                                                                const float* __restrict__ target, float lam_alpha,
                                                                float lam_texture, float* __restrict__ gW,
                                                                float* __restrict__ gTex, float* __restrict__ losses) {
  const float inv_p = 1.0f / (float)P;
  const float inv_3p = inv_p / 3.0f;
  float la = 0.f, lt = 0.f;
  for (int64_t p = (int64_t)blockIdx.x * kAuxThreads + threadIdx.x; p < P; p += (int64_t)gridDim.x * kAuxThreads) {
    const float* w = W + p * K;
    const float* x = tex + p * K * 3;
    float S = 0.f, A[3] = {0.f, 0.f, 0.f};
    for (int j = 0; j < K; ++j) {
      const float wj = w[j];
      S += wj;
      for (int c = 0; c < 3; ++c) A[c] = fmaf(wj, x[3 * j + c], A[c]);
    }
    la += 1.0f - S;
    float dr[3] = {0.f, 0.f, 0.f};  // dL_texture / dr_c
    float r[3] = {0.f, 0.f, 0.f};
    const bool has = S > 0.f;
    if (has) {
      for (int c = 0; c < 3; ++c) {
        r[c] = A[c] / S;
        const float e = target[3 * p + c] - r[c];
        lt += fabsf(e);
        dr[c] = e > 0.f ? -inv_3p : (e < 0.f ? inv_3p : 0.f);
      }
    }
    if (gW) {
      for (int j = 0; j < K; ++j) {
        float g = -lam_alpha * inv_p;
        if (has) {
          float t = 0.f;
          for (int c = 0; c < 3; ++c) t = fmaf(dr[c], x[3 * j + c] - r[c], t);
          g = fmaf(lam_texture, t / S, g);
        }
        gW[p * K + j] += g;
      }
    }
    if (gTex && has) {
      for (int j = 0; j < K; ++j) {
        const float f = lam_texture * w[j] / S;
        for (int c = 0; c < 3; ++c) gTex[(p * K + j) * 3 + c] += f * dr[c];
      }
    }
  }
  block_add(la * inv_p, losses + 0);
  block_add(lt * inv_3p, losses + 1);
}

__global__ __launch_bounds__(kAuxThreads) void aux_opacity_kernel(int64_t n, const float* __restrict__ o,
                                                                  float lam, float* __restrict__ g,
                                                                  float* __restrict__ losses) {
  const float inv_n = 1.0f / (float)n;
  float s = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * kAuxThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kAuxThreads) {
    s += o[i];
    if (g) g[i] += lam * inv_n;
  }
  block_add(s * inv_n, losses + 2);
}

struct LevelWeights {
  float w[kMaxLevels];  // s_l^-3
};

template <int TDT>
__device__ __forceinline__ float2 table_pair(const void* t, int64_t i) {
  if constexpr (TDT == NX_F32) {
    return reinterpret_cast<const float2*>(t)[i];
  } else {
    const uint32_t e = reinterpret_cast<const uint32_t*>(t)[i];
    if constexpr (TDT == NX_F16) {
      return make_float2(__half2float(__ushort_as_half((unsigned short)(e & 0xFFFFu))),
                         __half2float(__ushort_as_half((unsigned short)(e >> 16))));
    } else {
      return make_float2(__uint_as_float(e << 16), __uint_as_float(e & 0xFFFF0000u));
    }
  }
}

// One thread per table entry (F = 2 features).
template <int TDT>
__global__ __launch_bounds__(kAuxThreads) void aux_grid_kernel(int64_t n_entries, int log2_size, LevelWeights lw,
                                                               const void* __restrict__ table, float lam,
                                                               float2* __restrict__ g, float* __restrict__ losses) {
  float s = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * kAuxThreads + threadIdx.x; i < n_entries;
       i += (int64_t)gridDim.x * kAuxThreads) {
    const float2 h = table_pair<TDT>(table, i);
    const float c = lw.w[i >> log2_size];
    s = fmaf(c, fmaf(h.x, h.x, h.y * h.y), s);
    if (g) {
      float2 v = g[i];
      v.x = fmaf(2.0f * lam * c, h.x, v.x);
      v.y = fmaf(2.0f * lam * c, h.y, v.y);
      g[i] = v;
    }
  }
  block_add(s, losses + 3);
}

unsigned grid_for(int64_t n) {
  const int64_t b = (n + kAuxThreads - 1) / kAuxThreads;
  return (unsigned)(b < 2048 ? (b > 0 ? b : 1) : 2048);
}

}  // namespace

hipError_t launch_aux_losses(int64_t P, int K, const float* W, const float* tex, const float* target, float lam_alpha,
                             float lam_texture, float* gW, float* gTex, int64_t n, const float* opac, float lam_opacity,
                             float* g_opac, int feat_dtype, const void* table, int levels, int log2_size,
                             const float* level_scales, float lam_grid, float* g_table, float* losses, hipStream_t s) {
  hipLaunchKernelGGL(zero4_kernel, dim3(1), dim3(64), 0, s, losses);
  if (P > 0 && K > 0)
    hipLaunchKernelGGL(aux_pixel_kernel, dim3(grid_for(P)), dim3(kAuxThreads), 0, s, P, K, W, tex, target, lam_alpha,
                       lam_texture, gW, gTex, losses);
  if (n > 0)
    hipLaunchKernelGGL(aux_opacity_kernel, dim3(grid_for(n)), dim3(kAuxThreads), 0, s, n, opac, lam_opacity, g_opac,
                       losses);
  if (table && levels > 0) {
    LevelWeights lw{};
    for (int l = 0; l < levels; ++l) {
      const double sc = level_scales[l];
      lw.w[l] = (float)(1.0 / (sc * sc * sc));
    }
    const int64_t ne = (int64_t)levels << log2_size;
    float2* g2 = reinterpret_cast<float2*>(g_table);
    switch (feat_dtype) {
      case NX_F32:
        hipLaunchKernelGGL(aux_grid_kernel<NX_F32>, dim3(grid_for(ne)), dim3(kAuxThreads), 0, s, ne, log2_size, lw,
                           table, lam_grid, g2, losses);
        break;
      case NX_F16:
        hipLaunchKernelGGL(aux_grid_kernel<NX_F16>, dim3(grid_for(ne)), dim3(kAuxThreads), 0, s, ne, log2_size, lw,
                           table, lam_grid, g2, losses);
        break;
      default:
        hipLaunchKernelGGL(aux_grid_kernel<NX_BF16>, dim3(grid_for(ne)), dim3(kAuxThreads), 0, s, ne, log2_size, lw,
                           table, lam_grid, g2, losses);
        break;
    }
  }
  return hipGetLastError();
}

}  // namespace nx
