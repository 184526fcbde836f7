// Internal declarations shared by the HIP translation units of libnexels.
// Device helpers live here; every kernel is launched through a host
// function declared below so that the C-ABI layer stays free of kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nexels.h"

namespace nx {

// Constants of the method as this library reads them (the paper builds on
// the 3D Gaussian splatting rasteriser and leaves them implicit).
constexpr float kAlphaMin = 1.0f / 255.0f;   // skip intersections below this alpha
constexpr float kAlphaMax = 0.99f;           // alpha clamp
constexpr float kTMin = 1e-4f;               // stop before T would fall below this
constexpr float kSupport = 3.0f;             // hard kernel support |u|,|v| <= 3
constexpr int kTile = 16;                    // screen tile edge in pixels
constexpr double kMarginPx = 1.0;            // bounding-box margin for binning
constexpr uint32_t kPrime1 = 2654435761u;    // spatial hash primes (Instant-NGP)
constexpr uint32_t kPrime2 = 805459861u;

// Per-surfel record consumed by the collection pass: 5 float4.
//  [0] mx_int, my_int, hx, hy   pixel position of the projected centre split
//                               into an integer part and hx = 0.5 - frac
//  [1] p1x, p1y, p2x, p2y       numerators of u and v per pixel offset
//  [2] qx, qy, mz, opacity      denominator slope, centre depth, opacity
//  [3] gamma1, gamma2, r, g     kernel exponents and colour
//  [4] b, pad, pad, pad
// For a pixel offset (dx, dy) = (px + 0.5 - m_x, py + 0.5 - m_y):
//   den = 1 + dx qx + dy qy,  t = mz / den,
//   u = (dx p1x + dy p1y) / den,  v = (dx p2x + dy p2y) / den.
constexpr int kRecF4 = 5;
constexpr int kRecFloats = 4 * kRecF4;
// Record-gradient slots (float32, per surfel): d/d of
//   0 m_x, 1 m_y, 2 p1x, 3 p1y, 4 p2x, 5 p2y, 6 qx, 7 qy, 8 mz,
//   9 opacity, 10 gamma1, 11 gamma2, 12 r, 13 g, 14 b,
//   15 the blended error sum_p w_p E_p (not a gradient)
constexpr int kRecGrad = 16;

struct CamDev {
  double m[12];
  double fx, fy, cx, cy, near_z;
  int width, height, ntx, nty;
};

struct GridLevel {
  float scale;      // s_l
  float ofrac[3];   // frac(s_l * o): camera origin in level cells, fractional part
  int oint[3];      // floor(s_l * o)
  float kappa;      // (f / s_l)^2 / (2 pi), so Delta = -expm1(-kappa / D^2)
};

constexpr int kMaxLevels = 16;

struct GridDev {
  GridLevel lv[kMaxLevels];
  int levels, log2_size;
  float rot[9];     // camera-to-world rotation (R^T), row-major
  float fx, fy, cx, cy;
  int width, height;
};

struct ScatterCam;  // one camera's share of a joint hash-scatter launch (below)

// ---------------------------------------------------------------- launchers
// sh: colors holds 48 spherical-harmonics coefficients per surfel ([16][3])
// decoded along the direction from the camera centre, instead of RGB.
hipError_t launch_preprocess(const float* means, const float* quats, const float* scales, const float* opac,
                             const float* gammas, const float* colors, int sh, int64_t n, const CamDev& cam,
                             uint32_t* depth_keys, uint32_t* tile_counts, int4* rects, float4* records,
                             hipStream_t s);

hipError_t launch_preprocess_backward(const float* means, const float* quats, const float* scales,
                                      const float* colors, int sh, int64_t n, const CamDev& cam,
                                      const uint32_t* tile_counts, const float* rec_grad, float* g_means,
                                      float* g_quats, float* g_scales, float* g_opac, float* g_gammas,
                                      float* g_colors, float* g_blended, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs over bits [0, end_bit).
// keys/vals hold the input and receive the output; tmp_* are scratch of the
// same size; hist needs radix_hist_words(n) uint32 words. With n_dev the
// number of pairs is min(n, *n_dev), read on the device (n is then the
// capacity the launches are sized for, and no host synchronisation is needed).
size_t radix_hist_words(int64_t n);
hipError_t radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* tmp_keys, uint32_t* tmp_vals,
                            uint32_t* hist, int64_t n, int end_bit, hipStream_t s, const uint32_t* n_dev = nullptr);
hipError_t launch_copy_u32(const uint32_t* in, uint32_t* out, int64_t n, hipStream_t s,
                           const uint32_t* n_dev = nullptr);

hipError_t launch_iota(uint32_t* out, int64_t n, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* out, uint32_t value, int64_t n, hipStream_t s);
hipError_t launch_fill_f32(float* out, float value, int64_t n, hipStream_t s);
// offsets[i] = exclusive prefix sum of counts[order[i]]; offsets[n] = total.
hipError_t launch_gather_scan(const uint32_t* counts, const uint32_t* order, uint32_t* offsets,
                              uint32_t* block_sums, int64_t n, hipStream_t s);
size_t scan_block_words(int64_t n);
// Instances o >= cap are not written (cap = capacity of tile_keys / ids).
hipError_t launch_duplicate(const uint32_t* order, const uint32_t* offsets, const int4* rects, int64_t n,
                            int ntx, int64_t cap, uint32_t* tile_keys, uint32_t* ids, hipStream_t s);
hipError_t launch_tile_ranges(const uint32_t* tile_keys, int64_t n_inst, uint2* ranges, int n_tiles,
                              hipStream_t s, const uint32_t* n_dev = nullptr);

// Collection pass (one 16x16 tile per workgroup). batch: records staged in
// LDS per round, one of kRasterBatches.
constexpr int kRasterBatches[3] = {64, 128, 256};
constexpr int kRasterBatchDefault = 256;
hipError_t launch_raster_forward(int K, const float4* records, const uint32_t* sorted_ids, const uint2* ranges,
                                 const CamDev& cam, float* plain, int32_t* ids, float* weights, float* depths,
                                 float* t_final, uint32_t* n_iter, int batch, hipStream_t s);

hipError_t launch_raster_backward(int K, const float4* records, const uint32_t* sorted_ids, const uint2* ranges,
                                  const CamDev& cam, const float* plain, const int32_t* ids,
                                  const float* weights, const float* tex, const uint32_t* n_iter,
                                  const float* grad_image, const float* grad_weights, const float* grad_depth,
                                  const float* pixel_error, float* rec_grad, int batch, hipStream_t s);

struct MlpDev {
  const void* w[3];
  int in_dim, hidden;
};

// sh: the MLP head has 48 outputs, degree-3 SH coefficients decoded along
// the unit ray (colour = max(0, sum_k Y_k a_k + 0.5)), instead of a sigmoid RGB
// head of 3.
hipError_t launch_texture_forward(int K, int feat_dtype, int mlp_dtype, int sh, const GridDev& grid,
                                  const void* table, const MlpDev& mlp, const int32_t* ids, const float* depths,
                                  const float* weights, const float* plain, float* tex, float* image,
                                  int32_t* cells, uint32_t* relu_masks, float* features, hipStream_t s);

// Texture backward, first half: recompute features and MLP, back-propagate,
// accumulate the MLP weight gradients and the depth gradient, and write the
// gradient with respect to each level's interpolated feature pair (already
// scaled by Delta_l) to feat_grad (layout below).
hipError_t launch_texture_backward(int K, int feat_dtype, int mlp_dtype, int sh, const GridDev& grid,
                                   const void* table, const MlpDev& mlp, const int32_t* ids, const float* depths,
                                   const float* weights, const float* grad_image, const float* grad_tex,
                                   float2* feat_grad, float* g_mlp0, float* g_mlp1, float* g_mlp2,
                                   float* grad_depth, unsigned char* weight_ops, hipStream_t s);

// Workspace section for the backward's MLP operand slots in global memory
// (used for hidden width 128).
constexpr size_t kWeightOperandBytes = 256 * 1024;

// Texture backward, second half: distribute feat_grad over the 8 cell
// corners of every level and add the result into g_table, level by level:
// corner contributions are filed as records under buckets (fixed ranges of
// table entries), then one workgroup per bucket sums its records and updates
// that range of g_table (no floating-point global atomics).
// bin runs once per level over the blocks of every camera of the call (one
// joint launch), then reduce once per level. Records are filed in slabs: the
// bin launch runs `wgs` workgroups, each with a fixed share of the blocks,
// and workgroup w keeps the records of bucket b in its own slab of `slab`
// records at arena offset (w nb + b) slab; it ends by writing (slab start,
// records in it) to row w of the bucket's slab-table column
// (slab_table[b * n_rows + w]). A slab that fills up sends further records
// straight to the table with atomics (correct, slower). slab_cap > 0 shrinks
// the slabs and cas_rounds > 0 bounds the reduction's LDS compare-and-swap
// retries (then a global atomic), to exercise both fallbacks in tests; 0
// keeps the defaults. The n_cams cameras' n_blocks blocks are numbered camera
// after camera. One camera: cam0 (host) describes it and travels as the
// kernel's argument. Several: cams [n_cams] (device, written with
// launch_write_scatter_cam before the first level's launch) describe them.
hipError_t launch_write_scatter_cam(const ScatterCam& cam, ScatterCam* dst, hipStream_t s);
hipError_t launch_hash_scatter_bin(int K, const ScatterCam& cam0, const ScatterCam* cams, int n_cams, int64_t n_blocks,
                                   const GridDev& grid0, int level, float* g_table, int64_t n_rows, uint2* slab_table,
                                   uint16_t* rec_key, float2* rec_val, int64_t slab_cap, hipStream_t s);
hipError_t launch_hash_scatter_reduce(const GridDev& grid, int level, float* g_table, int64_t n_rows,
                                      int64_t n_blocks, const uint2* slab_table, const uint16_t* rec_key,
                                      const float2* rec_val, int cas_rounds, hipStream_t s);

// Auxiliary losses (L_alpha, L_texture over P pixels with K slots; L_opacity
// over n surfels; L_grid over the table): gradients scaled by the lambdas are
// added to gW [P,K], gTex [P,K,3], g_opac [n], g_table [levels][2^log2_size][2]
// (each may be null); losses[0..3] receive the unweighted values.
hipError_t launch_aux_losses(int64_t P, int K, const float* W, const float* tex, const float* target, float lam_alpha,
                             float lam_texture, float* gW, float* gTex, int64_t n, const float* opac, float lam_opacity,
                             float* g_opac, int feat_dtype, const void* table, int levels, int log2_size,
                             const float* level_scales, float lam_grid, float* g_table, float* losses, hipStream_t s);

// Adaptive density control. FPS: one cooperative launch of `grid`
// workgroups (fps_grid: the co-resident maximum, at most what n needs);
// best: n floats of scratch, slots: fps_slot_bytes(grid) bytes (16-byte
// aligned).
size_t fps_slot_bytes(int grid);
hipError_t fps_grid(int64_t n, int* grid);
hipError_t launch_fps(const float* pts, int64_t n, int64_t m, float* best, void* slots, int grid, int32_t* order,
                      float* d2, hipStream_t s);
// Split selection: chosen[i] = 1 for the k smallest keys err/draw (finite
// keys only); keys, ids, tmp_* are n words, hist radix_hist_words(n).
hipError_t launch_split_select(int64_t n, int64_t k, const float* err, const float* draws, uint32_t* keys,
                               uint32_t* ids, uint32_t* tmp_keys, uint32_t* tmp_ids, uint32_t* hist,
                               uint32_t* chosen, hipStream_t s);
// Split the chosen surfels and drop those with opacity < min_opacity;
// off1[n] + off2[n] (device) is the number written.
hipError_t launch_split_prune(int64_t n, const float* means, const float* quats, const float* scales,
                              const float* opac, const float* gammas, const float* colors, const uint32_t* chosen,
                              float min_opacity, uint32_t* keep1, uint32_t* keep2, uint32_t* off1, uint32_t* off2,
                              uint32_t* iota, uint32_t* scan_blocks, float* o_means, float* o_quats, float* o_scales,
                              float* o_opac, float* o_gammas, float* o_colors, int32_t* o_parent, hipStream_t s);

// Screen blocks of the hash scatter: bw x bh patches of 4x4 pixels with
// bw * bh * K = kScatUnits (patch, slot) units, i.e. at most 4096 corner
// records per block and level.
constexpr int kScatUnits = 32;
constexpr int kScatMaxBuckets = 2048;
struct ScatterGeom {
  int bw, bh, nbx, nby;
};
inline ScatterGeom scatter_geom(int width, int height, int K) {
  ScatterGeom g{1, 1, 0, 0};
  if (K <= 0) return g;
  const int np = K >= kScatUnits ? 1 : kScatUnits / K;
  while (g.bw * g.bw < np) g.bw *= 2;
  g.bh = np / g.bw > 0 ? np / g.bw : 1;
  const int npx = (width + 3) / 4, npy = (height + 3) / 4;
  g.nbx = (npx + g.bw - 1) / g.bw;
  g.nby = (npy + g.bh - 1) / g.bh;
  return g;
}
// Table entries per bucket (log2): 2^(log2_size - 8) clamped to [1, 2^13], so
// a level has 256 buckets up to 2^21 entries and at most 2048 at 2^24.
inline int scatter_bucket_log2(int log2_size) {
  const int b = log2_size - 8;
  return b < 0 ? 0 : (b > 13 ? 13 : b);
}
inline int scatter_buckets(int log2_size) { return 1 << (log2_size - scatter_bucket_log2(log2_size)); }
// Slabs of a bin launch: workgroups and records per (workgroup, bucket) slab,
// sized for 5/4 of the worst case (every corner of every sample a record)
// spread evenly over the buckets.
constexpr int kScatWorkgroups = 2048;       // up to 16 blocks each
constexpr int kScatWorkgroupsLarge = 3072;  // calls with more blocks
constexpr int kBlockRecords = 4096;  // at most 8 corner records per sample
struct ScatterSlabs {
  int64_t wgs, slab;
};
// Blocks of one camera (0 without texture slots).
inline int64_t scatter_blocks(int width, int height, int K) {
  const ScatterGeom g = scatter_geom(width, height, K);
  return K > 0 ? (int64_t)g.nbx * g.nby : 0;
}
// The same for a joint launch over nblk blocks of several cameras.
inline ScatterSlabs scatter_slabs_blocks(int64_t nblk, int nb) {
  ScatterSlabs r{0, 0};
  if (nblk <= 0) return r;
  r.wgs = nblk <= 16 * (int64_t)kScatWorkgroups ? (nblk < kScatWorkgroups ? nblk : kScatWorkgroups)
                                                  : kScatWorkgroupsLarge;
  const int64_t per_wg = (nblk + r.wgs - 1) / r.wgs;
  r.slab = (per_wg * kBlockRecords * 5 / 4 + nb - 1) / nb;
  return r;
}
// Arena records a joint launch over nblk blocks needs under any bucket count
// up to kScatMaxBuckets.
inline int64_t scatter_record_capacity_blocks(int64_t nblk) {
  const ScatterSlabs r = scatter_slabs_blocks(nblk, 1);
  return r.wgs * (r.slab + kScatMaxBuckets);
}

// One camera's share of a joint binning launch over all cameras of a call
// (device memory): its grid geometry, its depths [P,K] and per-level feature
// gradients, its block layout, and the index of its first block among the
// blocks of all cameras (cameras in call order).
struct ScatterCam {
  GridDev gd;
  const float* depths;
  const float2* feat_grad;
  int bw, bh, nbx, nby;
  int64_t blk0;
};

// The per-level feature gradients are stored for 4x4 pixel patches (row-major
// over the image, ragged at the right and bottom edges): element
// ((l * n_patches + q) * K + j) * 16 + c holds pixel c of patch q, slot j.
inline int64_t feat_grad_patches(int width, int height) {
  return (int64_t)((width + 3) / 4) * ((height + 3) / 4);
}
inline int64_t feat_grad_elems(int width, int height, int K) {
  return (int64_t)kMaxLevels * feat_grad_patches(width, height) * (K > 0 ? K : 0) * 16;
}

}  // namespace nx
