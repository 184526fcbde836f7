// Adaptive density control: farthest point sampling for initialisation, and
// the split / prune step of densification.
//
// Paper, supplementary, Adaptive Density Control:
//   * Initialisation: farthest point sampling orders the points so that each
//     next one maximises the distance to those already taken; the initial
//     scale of a point is its distance to the nearest earlier one.
//   * Densification: blended errors, normalised into probability weights,
//     draw a fraction of the surfels for splitting. With s1 >= s2 a surfel
//     becomes two with scales (s1/2, s2) and centres mu -/+ (s1/2) v1, every
//     other property copied; surfels whose opacity is below a threshold
//     (0.005) are then pruned.
// Choices the paper leaves open: FPS starts at point 0, compares squared
// distances evaluated in float32 as (dx dx + dy dy) + dz dz with every
// operation rounded, and breaks ties by the smallest index; the first point
// takes the second one's distance. The draw without replacement uses
// exponential clocks: surfel i gets the key e_i / w_i (e_i ~ Exp(1) supplied
// by the caller) and the smallest keys are drawn, which draws in proportion
// to w. The long axis is v2 when s2 > s1. The first child keeps the
// surfel's place among the survivors; second children follow all survivors
// in input order.
#include <hip/hip_cooperative_groups.h>

#include "nx_internal.h"

namespace nx {
namespace {

// One workgroup of 1024 per CU at most: every point taken costs a grid
// barrier and a read of every workgroup's candidate, both of which grow with
// the number of workgroups.
constexpr int kFpsThreads = 1024;
constexpr float kTaken = -1.0f;

__device__ __forceinline__ float dist2_rn(float ax, float ay, float az, float bx, float by, float bz) {
  const float dx = __fsub_rn(ax, bx), dy = __fsub_rn(ay, by), dz = __fsub_rn(az, bz);
  return __fadd_rn(__fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy)), __fmul_rn(dz, dz));
}

// Larger key = larger distance, then smaller index.
__device__ __forceinline__ unsigned long long fps_key(float d2, uint32_t i) {
  const uint32_t bits = d2 >= 0.0f ? __float_as_uint(d2) : 0u;
  return ((unsigned long long)bits << 32) | (unsigned long long)(0xFFFFFFFFu - i);
}

// A workgroup's candidate: its key and the point's coordinates, so that the
// winner's position needs no further load after the barrier.
struct alignas(16) FpsSlot {
  unsigned long long key;
  float x, y, z, pad;
};

struct FpsCand {
  unsigned long long key;
  float x, y, z;
};

__device__ __forceinline__ void take_max(FpsCand& a, unsigned long long k, float x, float y, float z) {
  if (k > a.key) {
    a.key = k;
    a.x = x;
    a.y = y;
    a.z = z;
  }
}

// The candidate with the largest key over the workgroup (every thread
// receives it).
__device__ FpsCand block_max(FpsCand v) {
  __shared__ FpsCand part[kFpsThreads / 64];
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long k = __shfl_xor(v.key, o, 64);
    const float x = __shfl_xor(v.x, o, 64), y = __shfl_xor(v.y, o, 64), z = __shfl_xor(v.z, o, 64);
    take_max(v, k, x, y, z);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) part[wave] = v;
  __syncthreads();
  FpsCand r = part[0];
  for (int w = 1; w < kFpsThreads / 64; ++w) take_max(r, part[w].key, part[w].x, part[w].y, part[w].z);
  __syncthreads();
  return r;
}

// Points held in registers per thread when n <= grid * kFpsThreads * this;
// larger inputs keep their distances in `best` (global memory) instead. The
// grid is sized so that n fits (fps_grid): each point taken costs one grid
// barrier, whose price grows with the number of workgroups, while the
// distance updates cost little.
constexpr int kFpsRegPoints = 8;

// One cooperative launch runs all m iterations: every workgroup updates the
// nearest-taken distances of its points against the point taken last, finds
// its best candidate, and posts it with its coordinates to a slot; after a
// grid barrier every workgroup reads all slots and takes the same winner.
// Slots alternate between two banks, so a bank is rewritten only after the
// barrier that follows its last read.
__global__ __launch_bounds__(kFpsThreads) void fps_kernel(const float* __restrict__ pts, int64_t n, int64_t m,
                                                          float* __restrict__ best, FpsSlot* slots,
                                                          int32_t* __restrict__ order, float* __restrict__ d2out) {
  namespace cg = cooperative_groups;
  cg::grid_group grid = cg::this_grid();
  const int G = gridDim.x;
  const int64_t stride = (int64_t)G * kFpsThreads;
  const int64_t first = (int64_t)blockIdx.x * kFpsThreads + threadIdx.x;
  const bool in_regs = n <= stride * kFpsRegPoints;
  float px[kFpsRegPoints], py[kFpsRegPoints], pz[kFpsRegPoints], pb[kFpsRegPoints];
  if (in_regs) {
#pragma unroll
    for (int r = 0; r < kFpsRegPoints; ++r) {
      const int64_t k = first + r * stride;
      const bool ok = k < n;
      px[r] = ok ? pts[3 * k] : 0.0f;
      py[r] = ok ? pts[3 * k + 1] : 0.0f;
      pz[r] = ok ? pts[3 * k + 2] : 0.0f;
      pb[r] = ok ? __int_as_float(0x7F800000) : kTaken;
    }
  } else {
    for (int64_t k = first; k < n; k += stride) best[k] = __int_as_float(0x7F800000);
  }
  uint32_t cur = 0;
  float cx = pts[0], cy = pts[1], cz = pts[2];
  if (blockIdx.x == 0 && threadIdx.x == 0) order[0] = 0;
  for (int64_t it = 0; it + 1 < m; ++it) {
    FpsCand mine{0ull, 0.0f, 0.0f, 0.0f};
    if (in_regs) {
#pragma unroll
      for (int r = 0; r < kFpsRegPoints; ++r) {
        const int64_t k = first + r * stride;
        float b = pb[r];
        if (k == (int64_t)cur) {
          b = kTaken;
        } else if (b != kTaken) {
          b = fminf(b, dist2_rn(px[r], py[r], pz[r], cx, cy, cz));
        }
        pb[r] = b;
        if (b != kTaken) take_max(mine, fps_key(b, (uint32_t)k), px[r], py[r], pz[r]);
      }
    } else {
      for (int64_t k = first; k < n; k += stride) {
        float b = best[k];
        const float x = pts[3 * k], y = pts[3 * k + 1], z = pts[3 * k + 2];
        if (k == (int64_t)cur) {
          b = kTaken;
        } else if (b != kTaken) {
          b = fminf(b, dist2_rn(x, y, z, cx, cy, cz));
        }
        best[k] = b;
        if (b != kTaken) take_max(mine, fps_key(b, (uint32_t)k), x, y, z);
      }
    }
    const FpsCand bk = block_max(mine);
    FpsSlot* bank = slots + (it & 1) * G;
    if (threadIdx.x == 0) bank[blockIdx.x] = FpsSlot{bk.key, bk.x, bk.y, bk.z, 0.0f};
    grid.sync();
    FpsCand w{0ull, 0.0f, 0.0f, 0.0f};
    for (int i = threadIdx.x; i < G; i += kFpsThreads) {
      const FpsSlot sl = bank[i];
      take_max(w, sl.key, sl.x, sl.y, sl.z);
    }
    w = block_max(w);
    // (a zero key cannot win while an untaken point remains, as m <= n)
    cur = w.key == 0ull ? 0u : 0xFFFFFFFFu - (uint32_t)(w.key & 0xFFFFFFFFull);
    cx = w.x;
    cy = w.y;
    cz = w.z;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      order[it + 1] = (int32_t)cur;
      d2out[it + 1] = __uint_as_float((uint32_t)(w.key >> 32));
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) d2out[0] = m > 1 ? d2out[1] : 0.0f;
}

// Draw keys: e / w as float32 bits (w <= 0: +inf, never drawn); values are the indices.
__global__ void split_keys_kernel(int64_t n, const float* __restrict__ err, const float* __restrict__ draws,
                                  uint32_t* __restrict__ keys, uint32_t* __restrict__ ids) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float w = err[i];
  keys[i] = w > 0.0f ? __float_as_uint(__fdiv_rn(draws[i], w)) : 0x7F800000u;
  ids[i] = (uint32_t)i;
}

// The first k entries of the sorted order with a finite key are drawn.
__global__ void split_mark_kernel(int64_t n, int64_t k, const uint32_t* __restrict__ keys,
                                  const uint32_t* __restrict__ ids, uint32_t* __restrict__ chosen) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n || r >= k) return;
  if (keys[r] < 0x7F800000u) chosen[ids[r]] = 1u;
}

__global__ void split_counts_kernel(int64_t n, const float* __restrict__ opac, float min_opacity,
                                   const uint32_t* __restrict__ chosen, uint32_t* __restrict__ keep1,
                                   uint32_t* __restrict__ keep2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t keep = opac[i] >= min_opacity ? 1u : 0u;
  keep1[i] = keep;
  keep2[i] = keep & chosen[i];
}

struct SurfelOut {
  float *means, *quats, *scales, *opac, *gammas, *colors;
  int32_t* parent;
};

__global__ void split_write_kernel(int64_t n, const float* __restrict__ means, const float* __restrict__ quats,
                                   const float* __restrict__ scales, const float* __restrict__ opac,
                                   const float* __restrict__ gammas, const float* __restrict__ colors,
                                   const uint32_t* __restrict__ chosen, const uint32_t* __restrict__ keep1,
                                   const uint32_t* __restrict__ off1, const uint32_t* __restrict__ off2,
                                   SurfelOut o) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !keep1[i]) return;
  const int64_t a = off1[i];
  float m[3] = {means[3 * i], means[3 * i + 1], means[3 * i + 2]};
  float s[2] = {scales[2 * i], scales[2 * i + 1]};
  const bool split = chosen[i] != 0u;
  float mb[3] = {m[0], m[1], m[2]};
  if (split) {
    // long axis: column 0 (v1) of the rotation if s1 >= s2, else column 1 (v2)
    // FP64 with every operation rounded (no contraction): the textbook
    // unit-quaternion matrix, then mu -/+ (s/2) axis, rounded to float32
    const double w = quats[4 * i], x = quats[4 * i + 1], y = quats[4 * i + 2], z = quats[4 * i + 3];
    const int which = s[0] >= s[1] ? 0 : 1;
    auto mul = [](double a, double b) { return __dmul_rn(a, b); };
    auto add = [](double a, double b) { return __dadd_rn(a, b); };
    auto sub = [](double a, double b) { return __dsub_rn(a, b); };
    double ax[3];
    if (which == 0) {
      ax[0] = sub(1.0, mul(2.0, add(mul(y, y), mul(z, z))));
      ax[1] = mul(2.0, add(mul(x, y), mul(w, z)));
      ax[2] = mul(2.0, sub(mul(x, z), mul(w, y)));
    } else {
      ax[0] = mul(2.0, sub(mul(x, y), mul(w, z)));
      ax[1] = sub(1.0, mul(2.0, add(mul(x, x), mul(z, z))));
      ax[2] = mul(2.0, add(mul(y, z), mul(w, x)));
    }
    const double half = 0.5 * (double)s[which];
    for (int c = 0; c < 3; ++c) {
      mb[c] = (float)add((double)m[c], mul(half, ax[c]));
      m[c] = (float)sub((double)m[c], mul(half, ax[c]));
    }
    s[which] = (float)half;
  }
  auto put = [&](int64_t at, const float* mu) {
    for (int c = 0; c < 3; ++c) o.means[3 * at + c] = mu[c];
    for (int c = 0; c < 4; ++c) o.quats[4 * at + c] = quats[4 * i + c];
    o.scales[2 * at] = s[0];
    o.scales[2 * at + 1] = s[1];
    o.opac[at] = opac[i];
    o.gammas[2 * at] = gammas[2 * i];
    o.gammas[2 * at + 1] = gammas[2 * i + 1];
    for (int c = 0; c < 3; ++c) o.colors[3 * at + c] = colors[3 * i + c];
    if (o.parent) o.parent[at] = (int32_t)i;
  };
  put(a, m);
  if (split) put((int64_t)off1[n] + off2[i], mb);
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

size_t fps_slot_bytes(int grid) { return sizeof(FpsSlot) * 2 * (size_t)grid; }

hipError_t fps_grid(int64_t n, int* grid) {
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fps_kernel, kFpsThreads, 0)) != hipSuccess) return e;
  if (per_cu < 1) return hipErrorCooperativeLaunchTooLarge;
  int64_t g = cus;  // at most one workgroup per CU (co-resident, as the grid barrier needs)
  const int64_t per_wg = (int64_t)kFpsThreads * kFpsRegPoints;
  const int64_t need = (n + per_wg - 1) / per_wg;  // as few as hold every point in registers
  if (g > need) g = need;
  *grid = (int)(g > 0 ? g : 1);
  return hipSuccess;
}

hipError_t launch_fps(const float* pts, int64_t n, int64_t m, float* best, void* slots_bytes, int grid, int32_t* order,
                      float* d2, hipStream_t s) {
  if (n <= 0 || m <= 0) return hipSuccess;
  FpsSlot* slots = static_cast<FpsSlot*>(slots_bytes);
  void* args[] = {(void*)&pts, (void*)&n, (void*)&m, (void*)&best, (void*)&slots, (void*)&order, (void*)&d2};
  return hipLaunchCooperativeKernel((const void*)fps_kernel, dim3(grid), dim3(kFpsThreads), args, 0, s);
}

hipError_t launch_split_select(int64_t n, int64_t k, const float* err, const float* draws, uint32_t* keys,
                               uint32_t* ids, uint32_t* tmp_keys, uint32_t* tmp_ids, uint32_t* hist,
                               uint32_t* chosen, hipStream_t s) {
  hipError_t e = launch_fill_u32(chosen, 0u, n, s);
  if (e != hipSuccess || n == 0 || k <= 0) return e;
  hipLaunchKernelGGL(split_keys_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, err, draws, keys, ids);
  if ((e = radix_sort_pairs(keys, ids, tmp_keys, tmp_ids, hist, n, 32, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(split_mark_kernel, dim3(blocks_for(n < k ? n : k)), dim3(256), 0, s, n, k, keys, ids, chosen);
  return hipGetLastError();
}

hipError_t launch_split_prune(int64_t n, const float* means, const float* quats, const float* scales,
                              const float* opac, const float* gammas, const float* colors, const uint32_t* chosen,
                              float min_opacity, uint32_t* keep1, uint32_t* keep2, uint32_t* off1, uint32_t* off2,
                              uint32_t* iota, uint32_t* scan_blocks, float* o_means, float* o_quats, float* o_scales,
                              float* o_opac, float* o_gammas, float* o_colors, int32_t* o_parent, hipStream_t s) {
  if (n == 0) {
    hipError_t e = launch_fill_u32(off1, 0u, 1, s);
    if (e != hipSuccess) return e;
    return launch_fill_u32(off2, 0u, 1, s);
  }
  hipLaunchKernelGGL(split_counts_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, opac, min_opacity, chosen, keep1,
                     keep2);
  hipError_t e = launch_iota(iota, n, s);
  if (e != hipSuccess) return e;
  if ((e = launch_gather_scan(keep1, iota, off1, scan_blocks, n, s)) != hipSuccess) return e;
  if ((e = launch_gather_scan(keep2, iota, off2, scan_blocks, n, s)) != hipSuccess) return e;
  SurfelOut o{o_means, o_quats, o_scales, o_opac, o_gammas, o_colors, o_parent};
  hipLaunchKernelGGL(split_write_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, means, quats, scales, opac, gammas,
                     colors, chosen, keep1, off1, off2, o);
  return hipGetLastError();
}

}  // namespace nx
