// Tile binning and ordering: prefix sums, instance emission, a stable LSD
// radix sort of (key, value) pairs, and per-tile ranges.
//
// Paper: surfels are sorted by the depth of their centres and composited per
// screen tile (Preliminaries, 2D Gaussian Splatting). Here the surfels are
// first sorted by depth key, the (tile, surfel) instances are emitted in that
// order, and a stable sort by tile index then yields, per tile, the surfels
// in (depth key, id) order.
//
// Radix sort: 8-bit digits, 4096 keys per block (4 waves x 16 rounds x 64).
// Each pass is an upsweep (per-block digit histograms), one exclusive scan
// over the digit-major histogram, and a downsweep that ranks keys within a
// wave by ballot matching on the digit bits; waves own contiguous key ranges
// and rounds run in order, so the sort is stable.
#include "nx_internal.h"

namespace nx {
namespace {

constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kRounds = 16;
constexpr int kWaveItems = kRounds * 64;
constexpr int kBlockItems = kSortWaves * kWaveItems;  // 4096
constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanBlock = kScanThreads * kScanItems;  // 1024

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

// Exclusive scan of 1024 values held 4 per thread (blocked). Returns the
// block total; each thread gets its exclusive prefix for its first item.
__device__ uint32_t block_excl_scan(uint32_t local_sum, uint32_t* s_wave, uint32_t* prefix_out) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t incl = wave_incl_scan(local_sum, lane);
  if (lane == 63) s_wave[wave] = incl;
  __syncthreads();
  uint32_t wbase = 0, total = 0;
  for (int w = 0; w < kScanThreads / 64; ++w) {
    const uint32_t v = s_wave[w];
    if (w < wave) wbase += v;
    total += v;
  }
  *prefix_out = wbase + incl - local_sum;
  __syncthreads();
  return total;
}

__global__ __launch_bounds__(kScanThreads) void scan_reduce_kernel(const uint32_t* __restrict__ in,
                                                                   const uint32_t* __restrict__ order, int64_t n,
                                                                   uint32_t* __restrict__ block_sums) {
  __shared__ uint32_t s_wave[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * kScanItems;
  uint32_t sum = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    if (i < n) sum += in[order ? order[i] : i];
  }
  uint32_t pre;
  const uint32_t total = block_excl_scan(sum, s_wave, &pre);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// Exclusive scan of block_sums[0..nb) in place; writes the grand total at [nb].
__global__ __launch_bounds__(kScanThreads) void scan_blocks_kernel(uint32_t* __restrict__ block_sums, int64_t nb) {
  __shared__ uint32_t s_wave[kScanThreads / 64];
  uint32_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += kScanBlock) {
    const int64_t base = b0 + threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t sum = 0;
    for (int k = 0; k < kScanItems; ++k) {
      v[k] = (base + k < nb) ? block_sums[base + k] : 0u;
      sum += v[k];
    }
    uint32_t pre;
    const uint32_t total = block_excl_scan(sum, s_wave, &pre);
    uint32_t run = carry + pre;
    for (int k = 0; k < kScanItems; ++k) {
      if (base + k < nb) block_sums[base + k] = run;
      run += v[k];
    }
    carry += total;
  }
  if (threadIdx.x == 0) block_sums[nb] = carry;
}

// `in` and `out` may be the same array (in-place scan).
__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(const uint32_t* in, const uint32_t* order,
                                                                  int64_t n, const uint32_t* block_sums,
                                                                  uint32_t* out, int64_t nb) {
  __shared__ uint32_t s_wave[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t sum = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    v[k] = (i < n) ? in[order ? order[i] : i] : 0u;
    sum += v[k];
  }
  uint32_t pre;
  block_excl_scan(sum, s_wave, &pre);
  uint32_t run = block_sums[blockIdx.x] + pre;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    if (i < n) out[i] = run;
    run += v[k];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = block_sums[nb];
}

// The element count is n, or min(n, *n_dev) when n_dev is given (a count
// that only the device knows, with n the capacity the launch was sized for).
__device__ __forceinline__ int64_t live_count(int64_t n, const uint32_t* n_dev) {
  if (!n_dev) return n;
  const int64_t d = (int64_t)*n_dev;
  return d < n ? d : n;
}

__global__ __launch_bounds__(kSortThreads) void radix_upsweep_kernel(const uint32_t* __restrict__ keys, int64_t n,
                                                                     const uint32_t* __restrict__ n_dev, int shift,
                                                                     int nblocks, uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kSortWaves][256];
  n = live_count(n, n_dev);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int d = tid; d < kSortWaves * 256; d += kSortThreads) (&h[0][0])[d] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kBlockItems + wave * kWaveItems;
  for (int r = 0; r < kRounds; ++r) {
    const int64_t i = base + r * 64 + lane;
    if (i < n) atomicAdd(&h[wave][(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  const uint32_t c = h[0][tid] + h[1][tid] + h[2][tid] + h[3][tid];
  hist[(int64_t)tid * nblocks + blockIdx.x] = c;
}

__global__ __launch_bounds__(kSortThreads) void radix_downsweep_kernel(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in, uint32_t* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out, const uint32_t* __restrict__ hist, int64_t n, const uint32_t* __restrict__ n_dev,
    int shift, int nblocks) {
  __shared__ uint32_t wcount[kSortWaves][256];
  n = live_count(n, n_dev);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int d = tid; d < kSortWaves * 256; d += kSortThreads) (&wcount[0][0])[d] = 0;
  __syncthreads();
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = (int64_t)blockIdx.x * kBlockItems + wave * kWaveItems;
  uint32_t k[kRounds], v[kRounds], rank[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int64_t i = base + r * 64 + lane;
    const bool valid = i < n;
    k[r] = valid ? keys_in[i] : 0u;
    v[r] = valid ? vals_in[i] : 0u;
  }
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int64_t i = base + r * 64 + lane;
    const bool valid = i < n;
    const uint32_t d = (k[r] >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t prior = (uint32_t)__popcll(peers & lt_mask);
    uint32_t before = 0;
    if (valid) before = wcount[wave][d];
    rank[r] = before + prior;
    __builtin_amdgcn_wave_barrier();
    if (valid && prior == 0) wcount[wave][d] = before + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  {
    uint32_t run = hist[(int64_t)tid * nblocks + blockIdx.x];
    for (int w = 0; w < kSortWaves; ++w) {
      const uint32_t c = wcount[w][tid];
      wcount[w][tid] = run;
      run += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int64_t i = base + r * 64 + lane;
    if (i < n) {
      const uint32_t d = (k[r] >> shift) & 255u;
      const uint32_t pos = wcount[wave][d] + rank[r];
      keys_out[pos] = k[r];
      vals_out[pos] = v[r];
    }
  }
}

__global__ void copy_u32_kernel(const uint32_t* __restrict__ in, uint32_t* __restrict__ out, int64_t n,
                                const uint32_t* __restrict__ n_dev) {
  n = live_count(n, n_dev);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = in[i];
}

__global__ void iota_kernel(uint32_t* out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (uint32_t)i;
}

__global__ void fill_u32_kernel(uint32_t* out, uint32_t value, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = value;
}

__global__ void fill_f32_kernel(float* out, float value, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = value;
}

// One wave per 64 consecutive surfels (in depth order): their instances
// form one contiguous range, which the wave writes with consecutive lanes on
// consecutive instances (coalesced, and long tile lists are shared by all
// lanes). Instance o of surfel j is tile (x0 + t mod w, y0 + t div w) with
// t = o - offsets[j], row-major over its rectangle. Instances at or past
// `cap` (the capacity of tile_keys / ids) are not written.
__global__ __launch_bounds__(256) void duplicate_kernel(const uint32_t* __restrict__ order,
                                                        const uint32_t* __restrict__ offsets,
                                                        const int4* __restrict__ rects, int64_t n, int ntx,
                                                        uint32_t cap, uint32_t* __restrict__ tile_keys,
                                                        uint32_t* __restrict__ ids) {
  __shared__ uint32_t soff[4][65];
  __shared__ uint32_t sid[4][64];
  __shared__ int4 srect[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i0 = ((int64_t)blockIdx.x * 4 + wave) * 64;
  if (i0 >= n) return;  // whole wave
  const int64_t i = i0 + lane;
  const bool valid = i < n;
  const uint32_t s = valid ? order[i] : 0u;
  soff[wave][lane] = offsets[valid ? i : n];
  if (lane == 0) soff[wave][64] = offsets[i0 + 64 < n ? i0 + 64 : n];
  sid[wave][lane] = s;
  srect[wave][lane] = valid ? rects[s] : make_int4(0, 0, -1, -1);
  // this wave's LDS rows are written and read by this wave only, and a
  // wave's LDS operations complete in issue order: only the compiler must
  // not move the reads above the writes
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
  __builtin_amdgcn_wave_barrier();
  const uint32_t base = soff[wave][0];
  const uint32_t end = soff[wave][64] < cap ? soff[wave][64] : cap;
  const uint32_t total = end > base ? end - base : 0u;
  // j: the last surfel whose range starts at or before o (non-empty: o < its
  // end). A lane's instances only move forward, 64 at a time, and a surfel
  // that covers thousands of tiles keeps every lane on it for many steps, so
  // the search starts from the previous j and is skipped while o is still
  // inside surfel j (one LDS read per step instead of six; the wave that
  // holds the largest surfels sets the kernel's duration).
  int j = 0;
  for (uint32_t k = lane; k < total; k += 64) {
    const uint32_t o = base + k;
    if (soff[wave][j + 1] <= o) {  // soff[wave][64] is the wave's end, above every o
      int lo = j + 1;
#pragma unroll
      for (int step = 32; step >= 1; step >>= 1)
        if (lo + step <= 63 && soff[wave][lo + step] <= o) lo += step;
      j = lo;
    }
    const int4 r = srect[wave][j];
    const uint32_t w = (uint32_t)(r.z - r.x + 1);
    const uint32_t t = o - soff[wave][j];
    const uint32_t ty = t / w, tx = t - ty * w;
    tile_keys[o] = (uint32_t)(((int)ty + r.y) * ntx + (int)tx + r.x);
    ids[o] = sid[wave][j];
  }
}

__global__ __launch_bounds__(256) void tile_ranges_kernel(const uint32_t* __restrict__ keys, int64_t n,
                                                          const uint32_t* __restrict__ n_dev,
                                                          uint2* __restrict__ ranges) {
  n = live_count(n, n_dev);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t t = keys[i];
  if (i == 0 || keys[i - 1] != t) ranges[t].x = (uint32_t)i;
  if (i == n - 1 || keys[i + 1] != t) ranges[t].y = (uint32_t)(i + 1);
}

inline unsigned grid1d(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

}  // namespace

size_t scan_block_words(int64_t n) { return (size_t)((n + kScanBlock - 1) / kScanBlock) + 1; }

size_t radix_hist_words(int64_t n) {
  const int64_t nb = (n + kBlockItems - 1) / kBlockItems;
  const int64_t h = 256 * (nb > 0 ? nb : 1);
  return (size_t)h + 1 + scan_block_words(h);
}

hipError_t launch_gather_scan(const uint32_t* counts, const uint32_t* order, uint32_t* offsets,
                              uint32_t* block_sums, int64_t n, hipStream_t s) {
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  if (nb == 0) return launch_fill_u32(offsets, 0u, 1, s);
  hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, counts, order, n, block_sums);
  hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(kScanThreads), 0, s, block_sums, nb);
  hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, counts, order, n, block_sums,
                     offsets, nb);
  return hipGetLastError();
}

hipError_t radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* tmp_keys, uint32_t* tmp_vals, uint32_t* hist,
                            int64_t n, int end_bit, hipStream_t s, const uint32_t* n_dev) {
  if (n <= 1 || end_bit <= 0) return hipSuccess;
  const int nblocks = (int)((n + kBlockItems - 1) / kBlockItems);
  const int64_t hn = 256 * (int64_t)nblocks;
  uint32_t* scan_tmp = hist + hn + 1;  // hist[hn] receives the grand total
  const int64_t snb = (hn + kScanBlock - 1) / kScanBlock;
  uint32_t *ki = keys, *vi = vals, *ko = tmp_keys, *vo = tmp_vals;
  int passes = 0;
  for (int shift = 0; shift < end_bit; shift += 8, ++passes) {
    hipLaunchKernelGGL(radix_upsweep_kernel, dim3(nblocks), dim3(kSortThreads), 0, s, ki, n, n_dev, shift, nblocks,
                       hist);
    hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)snb), dim3(kScanThreads), 0, s, hist, nullptr, hn,
                       scan_tmp);
    hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(kScanThreads), 0, s, scan_tmp, snb);
    // In-place exclusive scan of hist (each element read before it is written by the same thread).
    hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)snb), dim3(kScanThreads), 0, s, hist, nullptr, hn, scan_tmp,
                       hist, snb);
    hipLaunchKernelGGL(radix_downsweep_kernel, dim3(nblocks), dim3(kSortThreads), 0, s, ki, vi, ko, vo, hist, n,
                       n_dev, shift, nblocks);
    uint32_t* t;
    t = ki; ki = ko; ko = t;
    t = vi; vi = vo; vo = t;
  }
  if (passes & 1) {
    hipError_t e = launch_copy_u32(ki, keys, n, s, n_dev);
    if (e != hipSuccess) return e;
    e = launch_copy_u32(vi, vals, n, s, n_dev);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t launch_copy_u32(const uint32_t* in, uint32_t* out, int64_t n, hipStream_t s, const uint32_t* n_dev) {
  if (n == 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(copy_u32_kernel, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0, s, in, out, n,
                     n_dev);
  return hipGetLastError();
}

hipError_t launch_iota(uint32_t* out, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(iota_kernel, dim3(grid1d(n, 256)), dim3(256), 0, s, out, n);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* out, uint32_t value, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(grid1d(n, 256)), dim3(256), 0, s, out, value, n);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float* out, float value, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_f32_kernel, dim3(grid1d(n, 256)), dim3(256), 0, s, out, value, n);
  return hipGetLastError();
}

hipError_t launch_duplicate(const uint32_t* order, const uint32_t* offsets, const int4* rects, int64_t n, int ntx,
                            int64_t cap, uint32_t* tile_keys, uint32_t* ids, hipStream_t s) {
  if (n == 0 || cap <= 0) return hipSuccess;
  hipLaunchKernelGGL(duplicate_kernel, dim3(grid1d(n, 256)), dim3(256), 0, s, order, offsets, rects, n, ntx,
                     (uint32_t)(cap < 0xFFFFFFFFll ? cap : 0xFFFFFFFFll), tile_keys, ids);
  return hipGetLastError();
}

hipError_t launch_tile_ranges(const uint32_t* tile_keys, int64_t n_inst, uint2* ranges, int n_tiles,
                              hipStream_t s, const uint32_t* n_dev) {
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(ranges), 0u, 2 * (int64_t)n_tiles, s);
  if (e != hipSuccess || n_inst == 0) return e;
  hipLaunchKernelGGL(tile_ranges_kernel, dim3(grid1d(n_inst, 256)), dim3(256), 0, s, tile_keys, n_inst, n_dev,
                     ranges);
  return hipGetLastError();
}

}  // namespace nx
