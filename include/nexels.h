/*
 * nexels.h -- C ABI of the MI355X (gfx950) Nexels rendering library.
 *
 * The library renders neurally-textured surfels (Nexels, arXiv 2512.13796)
 * with two passes and differentiates them:
 *   collection pass  (Rendering, Collection Pass; eq. composite, eq. notexture):
 *                    per pixel, front-to-back alpha compositing of the
 *                    surfels' plain colours in centre-depth order, keeping the
 *                    K intersections of highest blending weight;
 *   texturing pass   (Rendering, Texturing Pass; eq. texture, eq. final):
 *                    hash-grid features at the K intersection points, scaled
 *                    by the down-weighting factor (eq. downweighting), decoded
 *                    by a bias-free ReLU MLP, and composited into the image.
 *
 * Conventions for every entry point:
 *   - Return value is an nx_status. Arguments are validated on the host
 *     before anything is launched; a failed call launches nothing and
 *     nx_last_error() describes the failure. A device fault from earlier
 *     asynchronous work is reported as NX_ERR_HIP by a later call.
 *   - "device" pointers must point to GPU memory of the current HIP device;
 *     "host" pointers to CPU memory. All device buffers are owned by the
 *     caller; the library allocates no device memory except a small pinned
 *     host word per context (and the fixed scratch array of
 *     nx_render_forward_noalloc, part of the loaded code object).
 *   - Arrays are dense and row-major; [a,b] means a rows of b elements.
 *   - Work is enqueued on the HIP stream passed as `stream` (NULL = the null
 *     stream). nx_render_forward synchronises that stream once per camera to
 *     read the number of tile instances; nx_render_forward_async and
 *     nx_render_backward do not synchronise.
 *   - Calls that share a workspace must not overlap.
 */
#ifndef NEXELS_H
#define NEXELS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NX_OK = 0,
  NX_ERR_INVALID = -1,     /* bad argument (null pointer, size, dtype, ...)  */
  NX_ERR_WORKSPACE = -2,   /* workspace too small; *workspace_required set  */
  NX_ERR_HIP = -3,         /* a HIP runtime call failed                     */
  NX_ERR_UNSUPPORTED = -4  /* valid but not implemented (e.g. K=3, F!=2)    */
} nx_status;

typedef enum { NX_F32 = 0, NX_F16 = 1, NX_BF16 = 2 } nx_dtype;

/* Most cameras one call renders. */
#define NX_MAX_CAMS 64

/* Surfel parameters, already activated (Representation, Geometry):
 * device pointers, float32.
 *   means     [n,3]  centres mu (world)
 *   quats     [n,4]  rotations (w,x,y,z), used as given (caller normalises);
 *                    R = [v1 v2 v3], v1/v2 span the surfel, v3 its normal
 *   scales    [n,2]  s1, s2 > 0 along v1, v2
 *   opacities [n]    in [0,1]
 *   gammas    [n,2]  generalised-Gaussian exponents, >= 1
 *   colors    [n,3]  plain (non-textured) RGB colour, or [n,48] SH
 *                    coefficients (nx_set_sh_degree)
 * Surfels with a non-finite parameter, a scale <= 0 or a centre at camera
 * depth <= near are culled (never drawn, zero gradient). */
typedef struct {
  const float *means, *quats, *scales, *opacities, *gammas, *colors;
  int64_t n;
} nx_surfels;

/* Pinhole camera (host struct). world_to_cam is the row-major 3x4 [R | t]
 * with x_cam = R x_world + t in the OpenCV frame (x right, y down, z
 * forward). Pixel (px, py) casts the ray through (px+0.5, py+0.5); its
 * parameter t is the camera-space depth. near is the near-plane depth. */
typedef struct {
  double world_to_cam[12];
  double fx, fy, cx, cy;
  double near_z;
  int32_t width, height;
} nx_camera;

/* Multiresolution hash grid (Preliminaries, Instant-NGP; supplementary
 * Implementation Details). table: device, [levels][1<<log2_size][feat] in
 * `dtype`. level_scales: HOST pointer, [levels] float32 scales s_l.
 * Supported: feat == 2, 1 <= levels <= 16, 4 <= log2_size <= 24. */
typedef struct {
  const void *table;
  nx_dtype dtype;
  int32_t levels, log2_size, feat;
  const float *level_scales;
} nx_hashgrid;

/* Texture MLP without biases (Results, implementation): w[i] is a device
 * [dims[i+1]][dims[i]] matrix in `dtype` (NX_F32 or NX_BF16). Hidden layers
 * use ReLU; the 3-channel RGB head a sigmoid, the 48-value SH head none (see
 * nx_set_sh_degree).
 * Supported: dims = {levels*feat (<= 32), 64 or 128, same, 3 or 48}. NX_F32 runs
 * on FP32 matrix cores, NX_BF16 on BF16 matrix cores with FP32 accumulation. */
typedef struct {
  const void *w[3];
  nx_dtype dtype;
  int32_t dims[4];
} nx_mlp;

/* Forward outputs (device, float32 unless noted), P = width*height:
 *   image   [P,3]    C = N + sum_j W_j Tex_j                    (eq. final)
 *   plain   [P,3]    N: plain colours of the unselected surfels (eq. notexture)
 *   ids     [P,K]    int32 ids of the selected surfels, compositing order, -1 empty
 *   weights [P,K]    blending weights W of the selected surfels (0 if empty)
 *   depths  [P,K]    intersection depths D (camera z, 0 if empty)
 *   t_final [P]      transmittance after the last composited surfel
 *   tex     [P,K,3]  decoded textures (0 if empty)
 *   n_iter  [P]      uint32, entries of the pixel's tile list the collection
 *                    pass consumed (bounds the backward replay)
 *   cells   [P,K,levels,3]  OPTIONAL (NULL = not written) int32 lattice cell
 *                    floor(s_l x) the texturing pass used per slot and level,
 *                    for inspecting the hash-cell decisions (0 for empty slots)
 *   relu_masks [P,K,2*hidden/32]  OPTIONAL (NULL = not written) uint32 bit
 *                    masks of the hidden units with a positive pre-activation,
 *                    layer 1 words then layer 2 words, bit i of word w for
 *                    unit 32 w + i (0 for empty slots)
 *   features [P,K,levels*feat]  OPTIONAL (NULL = not written) float32 MLP
 *                    inputs Delta_l * H_l(s_l x) per slot, level-major (feature
 *                    f of level l at 2 l + f), as computed before any rounding
 *                    to the MLP's storage type (0 for empty slots)
 *   n_instances      HOST array [n_cams] written by nx_render_forward: number
 *                    of (surfel, tile) pairs per camera; read by
 *                    nx_render_backward.
 * With n_cams > 1 every per-pixel array holds the cameras one after another
 * (camera c starts at pixel sum_{c'<c} width*height); the same holds for the
 * backward's grad_image / grad_weights / grad_tex. */
typedef struct {
  float *image, *plain;
  int32_t *ids;
  float *weights, *depths, *t_final, *tex;
  uint32_t *n_iter;
  int32_t *cells;
  uint32_t *relu_masks;
  float *features;
  int64_t *n_instances;
} nx_fwd_out;

/* Gradients, device float32, ACCUMULATED (+=) into caller-initialised
 * buffers: means [n,3], quats [n,4], scales [n,2], opacities [n],
 * gammas [n,2], colors [n,3], table [levels][1<<log2_size][feat] (always
 * float32 whatever the table's storage dtype), mlp[i] [dims[i+1]][dims[i]].
 * Any pointer may be NULL to skip that gradient.
 * Densification signal (supplementary, Densification: the blended errors of
 * Rota Bulo et al., summed over iterations): when both are non-NULL,
 * blended_error[i] (device, [n], +=) receives sum over pixels p of
 * w_{i,p} pixel_error[p], with w = alpha T the blending weight of every
 * surfel the collection pass composited at p (textured or not) and
 * pixel_error a caller-supplied device array [P] (cameras concatenated as
 * the forward's outputs), e.g. the pixel's L1 error. */
typedef struct {
  float *means, *quats, *scales, *opacities, *gammas, *colors;
  float *table;
  float *mlp[3];
  const float *pixel_error;
  float *blended_error;
} nx_grads;

/* Opaque context: fixed configuration plus one pinned host word. */
typedef struct nx_ctx nx_ctx;

/* Create a context. K in {0,1,2,4,8,16} is the number of textured
 * intersections per pixel (Collection Pass); tile must be 16. feat_dtype and
 * mlp_dtype are the storage dtypes later calls must use. */
int nx_create(nx_ctx **out, int32_t K, int32_t tile, nx_dtype feat_dtype, nx_dtype mlp_dtype);
int nx_destroy(nx_ctx *ctx);

/* Appearance (Representation, Appearance; Results: the experiments use
 * degree-3 harmonics, so the MLP has 48 outputs). degree -1 (the default):
 * nx_surfels.colors is [n,3] RGB and the MLP head has 3 outputs through a
 * sigmoid. degree 3: colors is
 * [n,48] spherical-harmonics coefficients in the layout [16][3] (coefficient
 * k of channel c at 3k + c), decoded along the unit direction from the camera
 * centre to the surfel centre as max(0, sum_k Y_k a_k + 0.5); the MLP head has
 * 48 outputs, the same coefficients for the texture, decoded the same way
 * along the pixel's unit ray direction; Y_k is the real SH basis with
 * orthonormal constants. Gradients: colors [n,48], and the surfel centre
 * also receives the gradient through the view direction. Other degrees:
 * NX_ERR_UNSUPPORTED. Set before the first forward; calls that share a
 * workspace must use one setting. */
int nx_set_sh_degree(nx_ctx *ctx, int32_t degree);

/* Workspace bytes for n_surfels surfels seen by n_cams cameras with at most
 * max_instances (surfel, tile) pairs per camera. The pair count depends on
 * the surfels themselves, so it cannot be known from the sizes alone: with
 * max_instances = 0 the result is the size for a single pair, enough for
 * nx_render_forward to count the pairs (it then
 * returns NX_ERR_WORKSPACE with the exact size in *workspace_required, after
 * one synchronisation per camera). The workspace starts with
 * the backward's hash-scatter scratch shared by the cameras (three record
 * arenas of about 10 records per sample, and their slab tables), then holds
 * one section per camera, one after another; the sections carry the
 * forward's sorted tile lists and per-surfel records to the backward. */
int nx_workspace_size(nx_ctx *ctx, int64_t n_surfels, const nx_camera *cams, int32_t n_cams,
                      int64_t max_instances, size_t *bytes);

/* The exact workspace size for these surfels and cameras (the pair counts
 * depend on the surfels, so nx_workspace_size with max_instances = 0 gives
 * only the size this call needs): runs the preprocess, the depth sort and the
 * pair count of each camera in `workspace` (at least
 * nx_workspace_size(ctx, n, cams + c, 1, 0) for every camera c; its contents
 * are overwritten), synchronises the stream once per camera, and stores in
 * *bytes the size nx_render_forward (or nx_render_forward_async with
 * max_instances = the largest count) needs, and in counts[c] (host array
 * [n_cams], may be NULL) camera c's number of (surfel, tile) pairs. */
int nx_workspace_size_exact(nx_ctx *ctx, const nx_surfels *surfels, const nx_camera *cams, int32_t n_cams,
                            void *workspace, size_t workspace_bytes, size_t *bytes, int64_t *counts, void *stream);

/* Collection pass, then texturing pass (Rendering), for each of the n_cams
 * cameras in cams (host array, 1 <= n_cams <= NX_MAX_CAMS, at most 2^30
 * pixels in total), one after another on the stream. If the workspace is too
 * small the call returns NX_ERR_WORKSPACE, stores a required size in
 * *workspace_required and leaves the outputs undefined; call again with a
 * workspace of at least that size (with several cameras the first estimate
 * may still be short: repeat until the call succeeds). On success
 * *workspace_required is the size the call used. */
int nx_render_forward(nx_ctx *ctx, const nx_surfels *surfels, const nx_camera *cams, int32_t n_cams,
                      const nx_hashgrid *grid, const nx_mlp *mlp, nx_fwd_out *out, void *workspace,
                      size_t workspace_bytes, size_t *workspace_required, void *stream);

/* nx_render_forward without any host synchronisation, so that it can be
 * captured in a HIP graph or queued back to back: every camera's section of
 * the workspace is laid out for max_instances (surfel, tile) pairs, the
 * instance count stays on the device, and the call returns as soon as the
 * work is queued. The workspace must hold nx_workspace_size(..., n_cams,
 * max_instances) bytes (NX_ERR_WORKSPACE otherwise, checked on the host).
 * out->n_instances[c] receives max_instances (the layout the backward reads).
 * A camera with more than max_instances pairs loses the pairs of its deepest
 * surfels (pairs are numbered in centre-depth order), and its outputs are
 * then wrong: read the true
 * counts with nx_instance_counts and call again with a larger bound when one
 * exceeds it. Outputs are otherwise bit-identical to nx_render_forward's. */
int nx_render_forward_async(nx_ctx *ctx, const nx_surfels *surfels, const nx_camera *cams, int32_t n_cams,
                            const nx_hashgrid *grid, const nx_mlp *mlp, nx_fwd_out *out, int64_t max_instances,
                            void *workspace, size_t workspace_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * nx_render_forward_async without a workspace argument. The call's
 * intermediate arrays live in a fixed array of NX_NOALLOC_SCRATCH_BYTES
 * inside the library (one per device, held from the library's first use on
 * that device until the process ends); the call allocates nothing and does
 * not synchronise. The caller still passes every output. Limit: the
 * forward-only layout for n_cams cameras at max_instances (surfel, tile)
 * pairs each (about 124 bytes per surfel plus 16 per pair, per camera) must
 * fit in the array, else NX_ERR_UNSUPPORTED with the size needed. Outputs
 * are bit-identical to nx_render_forward_async's (same overflow rule for a
 * camera with more than max_instances pairs); out->n_instances[c] receives
 * max_instances. Every call on one device shares that device's array and
 * leaves its contents behind: calls that overlap on one device (two
 * streams, two threads) race, and the array cannot serve a later
 * nx_render_backward (render with a workspace for training). Per-phase
 * timing records nothing during this call. */
#define NX_NOALLOC_SCRATCH_BYTES (64u << 20)
int nx_render_forward_noalloc(nx_ctx *ctx, const nx_surfels *surfels, const nx_camera *cams, int32_t n_cams,
                              const nx_hashgrid *grid, const nx_mlp *mlp, nx_fwd_out *out, int64_t max_instances,
                              void *stream);

/* True (surfel, tile) pair counts per camera of the last forward into
 * `workspace`, whose layout n_instances (as that forward left it in
 * out->n_instances) describes; synchronises `stream` first. counts: HOST
 * array [n_cams]. */
int nx_instance_counts(nx_ctx *ctx, int64_t n_surfels, const nx_camera *cams, int32_t n_cams,
                       const int64_t *n_instances, const void *workspace, size_t workspace_bytes, int64_t *counts,
                       void *stream);

/* Launch-shape tuning of the collection pass (the tiled rasteriser of the
 * Preliminaries section): each 16x16-pixel tile stages the records of its
 * surfels in LDS in rounds of `batch` records (64, 128 or 256; 256 unless
 * tuned). nx_autotune_raster times the collection-pass forward kernel of every
 * camera with each batch size, `reps` times after one warm-up (1 <= reps <=
 * 100), on the sorted tile lists a finished nx_render_forward (or _async)
 * left in `workspace` for these surfels and cameras (`out` as that call
 * returned it), and keeps the fastest for this context, keyed by K and the
 * cameras' sizes: later forward and backward calls over cameras of those
 * sizes use it. The kernel rewrites the collection pass's outputs in `out`
 * with the same values (the batch size does not change any result).
 * Synchronises the stream; *batch (host) receives the choice. */
int nx_autotune_raster(nx_ctx *ctx, const nx_surfels *surfels, const nx_camera *cams, int32_t n_cams,
                       const nx_fwd_out *out, const void *workspace, size_t workspace_bytes, int32_t reps,
                       int32_t *batch, void *stream);

/* Gradients of L through both passes given dL/dimage [P,3] (device) and the
 * optional dL/dweights [P,K] and dL/dtex [P,K,3] (device, NULL = zero), all
 * cameras concatenated as in the forward; the cameras' gradients add up in
 * grads. The call orders all its work after what stream already holds and
 * before what is queued on it later; part of it (the hash-grid gradient's
 * reductions, the collection-pass and preprocess backward) runs on two more
 * streams the context creates at its first backward (default priority; the
 * context then serves the device current at that time).
 * saved and workspace must be those of the matching forward call,
 * unmodified.
 * Discrete choices (stop, top-K, hash cell) are those the forward took.
 * Atomic accumulation makes results deterministic up to float32 summation
 * order. With a hash grid and K > 0 the call takes at most about 4e8 samples
 * (total pixels x K); beyond that it returns NX_ERR_UNSUPPORTED. */
int nx_render_backward(nx_ctx *ctx, const nx_surfels *surfels, const nx_camera *cams, int32_t n_cams,
                       const nx_hashgrid *grid, const nx_mlp *mlp, const nx_fwd_out *saved,
                       const void *workspace, size_t workspace_bytes, const float *grad_image,
                       const float *grad_weights, const float *grad_tex, const nx_grads *grads, void *stream);

/* Auxiliary losses of the optimisation (Optimization, Losses) and their
 * gradients, for the P pixels (cameras concatenated) of a forward with this
 * context's K:
 *   L_alpha   = 1/P sum_p (1 - sum_j W_pj)
 *   L_texture = 1/(3P) sum_p sum_c |GT_pc - sum_j W_pj Tex_pjc / sum_j W_pj|
 *               (pixels whose weights sum to 0 add nothing)
 *   L_opacity = 1/n sum_i o_i
 *   L_grid    = sum_l s_l^-3 sum_i sum_f H_lif^2 (the paper prints the term
 *               linear in H; it is read as this size-normalised weight decay)
 * weights [P,K], tex [P,K,3] (the forward's outputs), target [P,3],
 * opacities [n]: device float32; grid may be NULL (no L_grid). The gradient
 * of lambda_alpha L_alpha + lambda_texture L_texture + lambda_opacity
 * L_opacity + lambda_grid L_grid is ADDED (+=) to grad_weights [P,K] and
 * grad_tex [P,K,3] (pass them to nx_render_backward as dL/dW and dL/dTex),
 * grad_opacities [n] and grad_table (float32, the table's shape); any may be
 * NULL. losses: device float32 [4], set to the unweighted L_alpha,
 * L_texture, L_opacity, L_grid (workgroup partial sums added with atomics:
 * the last bits vary run to run). Enqueued on stream; no synchronisation. */
typedef struct {
  float alpha, texture, opacity, grid;
} nx_aux_lambdas;
int nx_aux_losses(nx_ctx *ctx, int64_t n_pixels, const float *weights, const float *tex, const float *target,
                  int64_t n_surfels, const float *opacities, const nx_hashgrid *grid, const nx_aux_lambdas *lambdas,
                  float *grad_weights, float *grad_tex, float *grad_opacities, float *grad_table, float *losses,
                  void *stream);

/* Adaptive density control (supplementary, Adaptive Density Control). */

/* Initialisation by farthest point sampling: order[0..m) receives the first
 * m points of the FPS order of points [n,3] (device float32), starting at
 * point 0, each next point maximising its distance to the points taken
 * before it; dist2[i] receives that squared distance (the squared initial
 * scale of point order[i]; dist2[0] = dist2[1]). Squared distances are
 * evaluated in float32 as (dx dx + dy dy) + dz dz with every operation
 * rounded; ties go to the smallest index. 1 <= m <= n < 2^31. order [m]
 * int32, dist2 [m] float32: device. One cooperative launch (a grid barrier
 * per point taken); the workspace needs nx_fps_workspace_size bytes. */
int nx_fps_workspace_size(int64_t n, size_t *bytes);
int nx_fps(nx_ctx *ctx, const float *points, int64_t n, int64_t m, int32_t *order, float *dist2, void *workspace,
           size_t workspace_bytes, void *stream);

/* Output of nx_densify: device float32 arrays of `capacity` surfels in the
 * layout of nx_surfels, and parent [capacity] int32 (the input surfel each
 * output came from). */
typedef struct {
  float *means, *quats, *scales, *opacities, *gammas, *colors;
  int32_t *parent;
  int64_t capacity;
} nx_surfels_out;

/* One densification step: draw n_split surfels for splitting with
 * probability in proportion to their blended errors (nx_grads.blended_error
 * summed over iterations), without replacement, by exponential clocks:
 * surfel i gets the key exp_draws[i] / blended_error[i] (float32; the caller
 * supplies exp_draws [n] >= 0, i.i.d. Exp(1)) and the n_split smallest finite
 * keys are drawn (surfels with error <= 0 never are; ties to the smaller
 * index). A drawn surfel with s1 >= s2 becomes two with scales (s1/2, s2) and
 * centres mu -/+ (s1/2) v1 (v2 and s2 when s2 > s1); rotation, opacity,
 * gammas and colour are copied. Then every surfel with opacity below
 * min_opacity (the paper uses 0.005) is dropped. Survivors keep their input
 * order (a split surfel's first child in its place); the second children
 * follow, in input order. out->capacity must be at least n + n_split; the
 * call synchronises the stream once to return the output count in *n_out
 * (host). The workspace needs nx_densify_workspace_size bytes. */
int nx_densify_workspace_size(int64_t n, size_t *bytes);
int nx_densify(nx_ctx *ctx, const nx_surfels *in, const float *blended_error, const float *exp_draws, int64_t n_split,
               float min_opacity, const nx_surfels_out *out, int64_t *n_out, void *workspace, size_t workspace_bytes,
               void *stream);

/* Byte offsets of the forward's intermediate arrays inside the workspace,
 * for inspection: depth keys [n] uint32 (float32 bits of the camera-space
 * centre depth), tile counts [n] uint32, tile rectangles [n,4] int32
 * (tx0,ty0,tx1,ty1), records [n,20] float32, sorted tile index [I] uint32,
 * sorted surfel id [I] uint32 (ordered by tile, then depth key, then id),
 * tile ranges [n_tiles,2] uint32 (start, end). */
typedef struct {
  size_t depth_keys, tile_counts, rects, records, sorted_tiles, sorted_ids, tile_ranges, total;
} nx_ws_layout;
int nx_workspace_layout(nx_ctx *ctx, int64_t n_surfels, const nx_camera *cams, int32_t n_cams,
                        int64_t n_instances, nx_ws_layout *layout);

/* Diagnostics: limits that force the hash-grid gradient's fallback paths,
 * which the default sizes use rarely. slab_records > 0 caps the records a
 * workgroup files per bucket slab (records beyond go straight to the table
 * with float atomics); cas_rounds > 0 caps the reduction's LDS
 * compare-and-swap retries (a record that loses them is added with a global
 * float atomic). 0 restores the default. Results stay the same up to float32
 * summation order; only speed changes. */
int nx_debug_limits(nx_ctx *ctx, int64_t slab_records, int32_t cas_rounds);

/* Per-phase timing for diagnostics and benchmarks. While enabled, every
 * kernel group a call launches (e.g. "raster_forward") is bracketed by two
 * hipEvents recorded on the call's stream; nx_timing_get syncs on them and
 * returns, for entry `index`, the phase name (static storage), the summed
 * milliseconds and the number of launches since the last reset. It returns
 * NX_ERR_INVALID when index is past the last entry. Not thread-safe. */
int nx_timing_enable(nx_ctx *ctx, int enabled);
int nx_timing_reset(nx_ctx *ctx);
int nx_timing_get(nx_ctx *ctx, int32_t index, const char **name, double *total_ms, int64_t *launches);

/* Message of the last failed call on this thread ("" if none). */
const char *nx_last_error(void);

/* ABI version (major*100 + minor). */
int nx_version(void);

#ifdef __cplusplus
}
#endif
#endif /* NEXELS_H */
