// C ABI of libnexels: argument validation, workspace layout and the launch
// sequence of the two rendering passes and their backward.
#include <math.h>
#include <stdio.h>

#include <map>

#include <mutex>
#include <string>
#include <vector>

#include "nx_internal.h"

struct nx_phase {
  const char* name;
  double ms;
  int64_t launches;
};

struct nx_pending {
  int phase;
  hipEvent_t a, b;
};

// Record arenas of the hash-grid gradient: level l is binned into arena
// l % kScatArenas while earlier levels are reduced on the side stream, so a
// bin waits only for the reduction of the level kScatArenas before it.
constexpr int kScatArenas = 3;

struct nx_ctx {
  int32_t K;
  int32_t tile;
  nx_dtype feat_dtype, mlp_dtype;
  int sh = 0;        // 1: spherical-harmonics appearance (48 coefficients per surfel and MLP head)
  int64_t debug_slab = 0;  // > 0: records per hash-scatter slab (forces the slab-full fallback)
  int debug_cas = 0;       // > 0: LDS compare-and-swap retries before a global atomic
  uint32_t* pinned;  // one host word for the instance-count readback
  bool timing;
  // Collection-pass records staged in LDS per round, chosen by
  // nx_autotune_raster per camera configuration (key: K and every camera's
  // size); configurations not tuned use the default. `batch` is the value
  // for the call in progress.
  std::map<std::string, int> tuned_batch;
  int batch = nx::kRasterBatchDefault;
  // The backward's extra streams (default priority) and the events that
  // order them with the call's stream: `side` runs each level's hash-scatter
  // reduction while the next level is binned, `side2` the collection-pass
  // and preprocess backward while the hash-grid gradient is formed. Created
  // at the first backward, on the device current then (a context serves one
  // device).
  hipStream_t side = nullptr, side2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_bin[kScatArenas] = {}, ev_red[kScatArenas] = {}, ev_tex = nullptr,
             ev_join2 = nullptr;
  std::vector<nx_phase> phases;
  std::vector<nx_pending> pending;
  std::vector<hipEvent_t> pool;
};

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

std::string camera_key(int K, const nx_camera* cams, int32_t n_cams) {
  std::string k = std::to_string(K);
  for (int32_t c = 0; c < n_cams; ++c) k += ":" + std::to_string(cams[c].width) + "x" + std::to_string(cams[c].height);
  return k;
}

// Selects the collection pass's LDS batch for a call over these cameras.
void select_batch(nx_ctx* ctx, const nx_camera* cams, int32_t n_cams) {
  const auto it = ctx->tuned_batch.find(camera_key(ctx->K, cams, n_cams));
  ctx->batch = it == ctx->tuned_batch.end() ? nx::kRasterBatchDefault : it->second;
}

#define NX_CHECK_HIP(expr)                                                                 \
  do {                                                                                     \
    hipError_t _e = (expr);                                                                \
    if (_e != hipSuccess) return fail(NX_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  // N-part
  size_t depth_keys, tile_counts, rects, records, sort_k, sort_v, sort_tk, sort_tv, offsets, scan_blocks;
  // fixed-size parts
  size_t tile_ranges, rec_grad, grad_depth, feat_grad, weight_ops;
  // I-part
  size_t hist, inst_tiles, inst_ids, inst_tmp_tiles, inst_tmp_ids;
  size_t total;
};

// fwd_only: leave out the arrays only the backward uses (record gradients,
// depth and feature gradients, weight operands).
Layout make_layout(int64_t n, const nx::CamDev& cd, int K, int64_t n_inst, bool fwd_only = false) {
  Layout L{};
  const int64_t n_pix = (int64_t)cd.width * cd.height;
  const int n_tiles = cd.ntx * cd.nty;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  const size_t nn = (size_t)(n > 0 ? n : 1);
  L.depth_keys = take(4 * nn);
  L.tile_counts = take(4 * nn);
  L.rects = take(16 * nn);
  L.records = take(sizeof(float) * nx::kRecFloats * nn);
  L.sort_k = take(4 * nn);
  L.sort_v = take(4 * nn);
  L.sort_tk = take(4 * nn);
  L.sort_tv = take(4 * nn);
  L.offsets = take(4 * (nn + 1));
  L.scan_blocks = take(4 * nx::scan_block_words((int64_t)nn));
  L.tile_ranges = take(8 * (size_t)n_tiles);
  L.rec_grad = take(fwd_only ? 0 : sizeof(float) * nx::kRecGrad * nn);
  L.grad_depth = take(fwd_only ? 0 : sizeof(float) * (size_t)(n_pix * (K > 0 ? K : 1)));
  L.feat_grad = take(fwd_only ? 0 : sizeof(float2) * (size_t)nx::feat_grad_elems(cd.width, cd.height, K));
  L.weight_ops = take(fwd_only || K == 0 ? 0 : nx::kWeightOperandBytes);
  const int64_t ni = n_inst > 0 ? n_inst : 1;
  const int64_t hist_n = ni > (int64_t)nn ? ni : (int64_t)nn;
  L.hist = take(4 * nx::radix_hist_words(hist_n));
  L.inst_tiles = take(4 * (size_t)ni);
  L.inst_ids = take(4 * (size_t)ni);
  L.inst_tmp_tiles = take(4 * (size_t)ni);
  L.inst_tmp_ids = take(4 * (size_t)ni);
  L.total = o;
  return L;
}

// The hash-grid scatter's record arenas and slab tables are shared by the
// cameras of a call (every level is reduced once for all of them); they sit
// at the start of the workspace, before the per-camera sections.
struct SharedLayout {
  // kScatArenas arenas: level l files into arena l % kScatArenas while earlier levels are reduced
  size_t rec_key[kScatArenas], rec_val[kScatArenas], slab_table[kScatArenas], cams, total;
  int64_t capacity;  // records per arena
  int64_t rows;      // slab-table rows (workgroups of the joint bin launch)
  int64_t blocks;    // bin blocks over all cameras
};

SharedLayout make_shared_layout(const nx_camera* cams, int32_t n_cams, int K) {
  SharedLayout S{};
  for (int32_t c = 0; c < n_cams && K > 0; ++c) S.blocks += nx::scatter_blocks(cams[c].width, cams[c].height, K);
  if (S.blocks > 0) {
    S.capacity = nx::scatter_record_capacity_blocks(S.blocks);
    S.rows = nx::scatter_slabs_blocks(S.blocks, 1).wgs;
  }
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  for (int a = 0; a < kScatArenas; ++a) {
    S.rec_key[a] = take(sizeof(uint16_t) * (size_t)S.capacity);
    S.rec_val[a] = take(sizeof(float2) * (size_t)S.capacity);
    S.slab_table[a] = take(sizeof(uint2) * (size_t)S.rows * nx::kScatMaxBuckets);
  }
  S.cams = take(S.blocks > 0 ? sizeof(nx::ScatterCam) * (size_t)n_cams : 0);
  S.total = o;
  return S;
}

bool finite_d(double x) { return isfinite(x); }

int check_ctx(const nx_ctx* ctx) {
  if (!ctx) return fail(NX_ERR_INVALID, "ctx is NULL");
  return NX_OK;
}

int check_camera(const nx_camera* cams, int32_t n_cams) {
  if (!cams) return fail(NX_ERR_INVALID, "cams is NULL");
  if (n_cams < 1) return fail(NX_ERR_INVALID, "n_cams must be at least 1");
  if (n_cams > NX_MAX_CAMS) return fail(NX_ERR_UNSUPPORTED, "n_cams exceeds NX_MAX_CAMS");
  int64_t total = 0;
  for (int32_t k = 0; k < n_cams; ++k) {
    const nx_camera& c = cams[k];
    if (c.width <= 0 || c.height <= 0) return fail(NX_ERR_INVALID, "camera width/height must be positive");
    if ((int64_t)c.width * c.height > (int64_t)1 << 28) return fail(NX_ERR_UNSUPPORTED, "image larger than 2^28 px");
    total += (int64_t)c.width * c.height;
    for (int i = 0; i < 12; ++i)
      if (!finite_d(c.world_to_cam[i])) return fail(NX_ERR_INVALID, "camera matrix not finite");
    if (!(c.fx > 0 && c.fy > 0 && finite_d(c.fx) && finite_d(c.fy) && finite_d(c.cx) && finite_d(c.cy)))
      return fail(NX_ERR_INVALID, "camera intrinsics invalid");
    if (!(c.near_z > 0 && finite_d(c.near_z))) return fail(NX_ERR_INVALID, "near_z must be positive");
  }
  if (total > (int64_t)1 << 30) return fail(NX_ERR_UNSUPPORTED, "more than 2^30 pixels in one call");
  return NX_OK;
}

int check_surfels(const nx_surfels* s) {
  if (!s) return fail(NX_ERR_INVALID, "surfels is NULL");
  if (s->n < 0) return fail(NX_ERR_INVALID, "negative surfel count");
  if (s->n >= ((int64_t)1 << 31)) return fail(NX_ERR_UNSUPPORTED, "more than 2^31-1 surfels");
  if (s->n > 0 && (!s->means || !s->quats || !s->scales || !s->opacities || !s->gammas || !s->colors))
    return fail(NX_ERR_INVALID, "a surfel parameter pointer is NULL");
  return NX_OK;
}

int check_grid_mlp(const nx_ctx* ctx, const nx_hashgrid* g, const nx_mlp* m) {
  if (ctx->K == 0) return NX_OK;  // no texturing pass
  if (!g || !m) return fail(NX_ERR_INVALID, "grid or mlp is NULL");
  if (!g->table || !g->level_scales) return fail(NX_ERR_INVALID, "grid table or level_scales is NULL");
  if (g->dtype != ctx->feat_dtype) return fail(NX_ERR_INVALID, "grid dtype differs from the context's feat_dtype");
  if (g->feat != 2) return fail(NX_ERR_UNSUPPORTED, "only feat == 2 is supported");
  if (g->levels < 1 || g->levels > 16) return fail(NX_ERR_UNSUPPORTED, "levels must be in [1, 16]");
  if (g->log2_size < 4 || g->log2_size > 24) return fail(NX_ERR_UNSUPPORTED, "log2_size must be in [4, 24]");
  for (int l = 0; l < g->levels; ++l)
    if (!(g->level_scales[l] > 0.0f) || !isfinite(g->level_scales[l]))
      return fail(NX_ERR_INVALID, "level scales must be positive and finite");
  if (m->dtype != ctx->mlp_dtype) return fail(NX_ERR_INVALID, "mlp dtype differs from the context's mlp_dtype");
  if (!m->w[0] || !m->w[1] || !m->w[2]) return fail(NX_ERR_INVALID, "an MLP weight pointer is NULL");
  if (m->dims[0] != g->levels * g->feat) return fail(NX_ERR_INVALID, "mlp dims[0] must equal levels * feat");
  if (m->dims[1] != m->dims[2] || (m->dims[1] != 64 && m->dims[1] != 128))
    return fail(NX_ERR_UNSUPPORTED, "hidden widths must be equal and 64 or 128");
  if (m->dims[3] != (ctx->sh ? 48 : 3))
    return fail(NX_ERR_UNSUPPORTED, ctx->sh ? "the MLP head must have 48 outputs (degree-3 SH coefficients)"
                                            : "the MLP head must have 3 outputs");
  return NX_OK;
}

nx::CamDev make_cam(const nx_camera& c) {
  nx::CamDev d;
  for (int i = 0; i < 12; ++i) d.m[i] = c.world_to_cam[i];
  d.fx = c.fx;
  d.fy = c.fy;
  d.cx = c.cx;
  d.cy = c.cy;
  d.near_z = c.near_z;
  d.width = c.width;
  d.height = c.height;
  d.ntx = (c.width + nx::kTile - 1) / nx::kTile;
  d.nty = (c.height + nx::kTile - 1) / nx::kTile;
  return d;
}

nx::GridDev make_grid(const nx_camera& c, const nx_hashgrid* g) {
  nx::GridDev d{};
  const double* m = c.world_to_cam;
  // camera centre in world: o = -R^T t
  double o[3];
  for (int k = 0; k < 3; ++k) o[k] = -(m[0 + k] * m[3] + m[4 + k] * m[7] + m[8 + k] * m[11]);
  d.levels = g ? g->levels : 0;
  d.log2_size = g ? g->log2_size : 0;
  for (int l = 0; l < d.levels; ++l) {
    const double s = g->level_scales[l];
    d.lv[l].scale = g->level_scales[l];
    for (int k = 0; k < 3; ++k) {
      const double so = s * o[k];
      const double fl = floor(so);
      d.lv[l].oint[k] = (int)fl;
      d.lv[l].ofrac[k] = (float)(so - fl);
    }
    const double r = c.fx / s;
    d.lv[l].kappa = (float)(r * r / (2.0 * M_PI));
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) d.rot[3 * i + j] = (float)m[4 * j + i];
  d.fx = (float)c.fx;
  d.fy = (float)c.fy;
  d.cx = (float)c.cx;
  d.cy = (float)c.cy;
  d.width = c.width;
  d.height = c.height;
  return d;
}

int tile_bits(int n_tiles) {
  int b = 0;
  while (b < 31 && ((int64_t)1 << b) < n_tiles) ++b;
  return b;
}

hipEvent_t take_event(nx_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  // timing only: no system-scope fence (no cache writeback and invalidate
  // around the timed launches)
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

int phase_index(nx_ctx* c, const char* name) {
  for (size_t i = 0; i < c->phases.size(); ++i)
    if (c->phases[i].name == name) return (int)i;
  c->phases.push_back({name, 0.0, 0});
  return (int)c->phases.size() - 1;
}

// Brackets the launches of one phase with events when timing is enabled.
struct PhaseTimer {
  nx_ctx* c;
  hipStream_t s;
  int phase = -1;
  hipEvent_t a = nullptr;
  PhaseTimer(nx_ctx* ctx, const char* name, hipStream_t stream) : c(ctx), s(stream) {
    if (!c->timing) return;
    a = take_event(c);
    if (a && hipEventRecord(a, s) == hipSuccess) phase = phase_index(c, name);
  }
  ~PhaseTimer() {
    if (phase < 0) return;
    hipEvent_t b = take_event(c);
    if (b && hipEventRecord(b, s) == hipSuccess) c->pending.push_back({phase, a, b});
  }
};

// The backward's extra streams and their events, created once per context.
int side_streams(nx_ctx* c) {
  if (c->side) return NX_OK;
  hipStream_t st[2] = {nullptr, nullptr};
  for (hipStream_t& x : st) {
    const hipError_t err = hipStreamCreateWithFlags(&x, hipStreamNonBlocking);
    if (err != hipSuccess) {
      if (st[0]) (void)hipStreamDestroy(st[0]);
      return fail(NX_ERR_HIP, std::string("hipStreamCreateWithFlags: ") + hipGetErrorString(err));
    }
  }
  std::vector<hipEvent_t*> evs = {&c->ev_fork, &c->ev_join, &c->ev_tex, &c->ev_join2};
  for (int a = 0; a < kScatArenas; ++a) {
    evs.push_back(&c->ev_bin[a]);
    evs.push_back(&c->ev_red[a]);
  }
  for (hipEvent_t* e : evs) {
    // ordering between streams of one device: a device-scope release is enough
    const hipError_t err = hipEventCreateWithFlags(e, hipEventDisableTiming | hipEventReleaseToDevice);
    if (err != hipSuccess) {
      (void)hipStreamDestroy(st[0]);
      (void)hipStreamDestroy(st[1]);
      return fail(NX_ERR_HIP, std::string("hipEventCreateWithFlags: ") + hipGetErrorString(err));
    }
  }
  c->side = st[0];
  c->side2 = st[1];
  return NX_OK;
}

template <typename T>
T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + off);
}
template <typename T>
const T* at(const void* base, size_t off) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off);
}

// The outputs of the camera whose pixels start at pixel offset pix in the
// concatenated arrays.
nx_fwd_out camera_slice(const nx_ctx* ctx, const nx_hashgrid* grid, const nx_mlp* mlp, const nx_fwd_out& o,
                        int64_t pix) {
  const int64_t K = ctx->K > 0 ? ctx->K : 0;
  nx_fwd_out c = o;
  c.image = o.image + 3 * pix;
  c.plain = o.plain + 3 * pix;
  c.t_final = o.t_final + pix;
  c.n_iter = o.n_iter + pix;
  if (o.ids) c.ids = o.ids + K * pix;
  if (o.weights) c.weights = o.weights + K * pix;
  if (o.depths) c.depths = o.depths + K * pix;
  if (o.tex) c.tex = o.tex + 3 * K * pix;
  if (o.cells && grid) c.cells = o.cells + (int64_t)3 * grid->levels * K * pix;
  if (o.relu_masks && mlp) c.relu_masks = o.relu_masks + (int64_t)2 * (mlp->dims[1] / 32) * K * pix;
  if (o.features && grid) c.features = o.features + (int64_t)grid->levels * grid->feat * K * pix;
  return c;
}

// Collection pass up to the instance scan: per-surfel keys, counts,
// rectangles and records, the depth sort, and the exclusive scan of the tile
// counts in depth order (offsets[n] = number of instances, on the device).
int forward_prefix(nx_ctx* ctx, const nx_surfels* surfels, const nx::CamDev& cd, void* ws, const Layout& L0,
                   hipStream_t s) {
  const int64_t n = surfels->n;

  uint32_t* depth_keys = at<uint32_t>(ws, L0.depth_keys);
  uint32_t* counts = at<uint32_t>(ws, L0.tile_counts);
  int4* rects = at<int4>(ws, L0.rects);
  float4* records = at<float4>(ws, L0.records);
  {
  PhaseTimer pt(ctx, "preprocess", s);
  NX_CHECK_HIP(nx::launch_preprocess(surfels->means, surfels->quats, surfels->scales, surfels->opacities,
                                     surfels->gammas, surfels->colors, ctx->sh, n, cd, depth_keys, counts, rects,
                                     records, s));
  }
  uint32_t* sk = at<uint32_t>(ws, L0.sort_k);
  uint32_t* sv = at<uint32_t>(ws, L0.sort_v);
  uint32_t* offsets = at<uint32_t>(ws, L0.offsets);
  if (n > 0) {
    PhaseTimer pt(ctx, "depth_sort", s);
    NX_CHECK_HIP(nx::launch_copy_u32(depth_keys, sk, n, s));
    NX_CHECK_HIP(nx::launch_iota(sv, n, s));
    // The I-part is not laid out yet: the histogram for the depth sort uses the
    // instance area, which is at least as large as the N-sized histogram.
    NX_CHECK_HIP(nx::radix_sort_pairs(sk, sv, at<uint32_t>(ws, L0.sort_tk), at<uint32_t>(ws, L0.sort_tv),
                                      at<uint32_t>(ws, L0.hist), n, 32, s));
  }
  {
    PhaseTimer pt(ctx, "instance_scan", s);
    NX_CHECK_HIP(nx::launch_gather_scan(counts, sv, offsets, at<uint32_t>(ws, L0.scan_blocks), n, s));
  }
  return NX_OK;
}

// One camera of nx_render_forward: out points at this camera's slices of the
// outputs, workspace at its section. With cap < 0 the call reads the
// instance count back (one synchronisation) and lays the section out for
// exactly that many; *need receives the section size this camera requires
// so far. With cap >= 0 the section is laid out for cap instances, nothing
// is read back, and instances past cap are dropped (the device keeps the
// true count at offsets[n]).
int forward_one(nx_ctx* ctx, const nx_surfels* surfels, const nx_camera& cam, const nx_hashgrid* grid,
                const nx_mlp* mlp, const nx_fwd_out* out, void* workspace, size_t workspace_bytes, size_t* need,
                int64_t* n_inst_out, hipStream_t s, int64_t cap = -1, bool fwd_only = false) {
  const int K = ctx->K;
  const nx::CamDev cd = make_cam(cam);
  const int n_tiles = cd.ntx * cd.nty;
  const int64_t n = surfels->n;
  const Layout L0 = make_layout(n, cd, K, cap >= 0 ? cap : 0, fwd_only);
  *need = L0.total;
  if (!workspace || workspace_bytes < L0.total) return fail(NX_ERR_WORKSPACE, "workspace too small");
  void* ws = workspace;
  int r = forward_prefix(ctx, surfels, cd, ws, L0, s);
  if (r != NX_OK) return r;
  uint32_t* sv = at<uint32_t>(ws, L0.sort_v);
  uint32_t* offsets = at<uint32_t>(ws, L0.offsets);
  int4* rects = at<int4>(ws, L0.rects);
  float4* records = at<float4>(ws, L0.records);
  int64_t n_inst;
  const uint32_t* n_dev = nullptr;
  if (cap < 0) {
    NX_CHECK_HIP(hipMemcpyAsync(ctx->pinned, offsets + n, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    NX_CHECK_HIP(hipStreamSynchronize(s));
    n_inst = (int64_t)ctx->pinned[0];
  } else {
    n_inst = cap;
    n_dev = offsets + n;
  }
  const Layout L = make_layout(n, cd, K, n_inst, fwd_only);
  *n_inst_out = n_inst;
  *need = L.total;
  if (workspace_bytes < L.total) return fail(NX_ERR_WORKSPACE, "workspace too small for the tile instances");

  uint32_t* it = at<uint32_t>(ws, L.inst_tiles);
  uint32_t* iid = at<uint32_t>(ws, L.inst_ids);
  {
    PhaseTimer pt(ctx, "duplicate", s);
    NX_CHECK_HIP(nx::launch_duplicate(sv, offsets, rects, n, cd.ntx, n_inst, it, iid, s));
  }
  {
  PhaseTimer pt(ctx, "tile_sort", s);
  NX_CHECK_HIP(nx::radix_sort_pairs(it, iid, at<uint32_t>(ws, L.inst_tmp_tiles), at<uint32_t>(ws, L.inst_tmp_ids),
                                    at<uint32_t>(ws, L.hist), n_inst, tile_bits(n_tiles), s, n_dev));
  }
  uint2* ranges = at<uint2>(ws, L.tile_ranges);
  {
    PhaseTimer pt(ctx, "tile_ranges", s);
    NX_CHECK_HIP(nx::launch_tile_ranges(it, n_inst, ranges, n_tiles, s, n_dev));
  }
  {
  PhaseTimer pt(ctx, "raster_forward", s);
  NX_CHECK_HIP(nx::launch_raster_forward(K, records, iid, ranges, cd, out->plain, out->ids, out->weights,
                                         out->depths, out->t_final, out->n_iter, ctx->batch, s));
  }
  nx::GridDev gd = make_grid(cam, grid);
  nx::MlpDev md{};
  if (K > 0) {
    md.w[0] = mlp->w[0];
    md.w[1] = mlp->w[1];
    md.w[2] = mlp->w[2];
    md.in_dim = mlp->dims[0];
    md.hidden = mlp->dims[1];
  }
  {
  PhaseTimer pt(ctx, "texture_forward", s);
  NX_CHECK_HIP(nx::launch_texture_forward(K, ctx->feat_dtype, ctx->mlp_dtype, ctx->sh, gd, K > 0 ? grid->table : nullptr, md,
                                          out->ids, out->depths, out->weights, out->plain, out->tex, out->image,
                                          out->cells, out->relu_masks, out->features, s));
  }
  return NX_OK;
}

// One camera of nx_render_backward: saved, grad_* point at this camera's
// slices, workspace at its section (laid out for n_inst instances). Part 0:
// zero the record gradients, texture backward; part 1 (after part 0 of every
// camera): collection-pass and preprocess backward.
int backward_one(nx_ctx* ctx, const nx_surfels* surfels, const nx_camera& cam, const nx_hashgrid* grid,
                 const nx_mlp* mlp, const nx_fwd_out* saved, int64_t n_inst, void* workspace,
                 const float* grad_image, const float* grad_weights, const float* grad_tex, const nx_grads* grads,
                 const float* pixel_error, hipStream_t s, int part) {
  const int K = ctx->K;
  const nx::CamDev cd = make_cam(cam);
  const int64_t n = surfels->n;
  const Layout L = make_layout(n, cd, K, n_inst);
  void* ws = workspace;
  float* rec_grad = at<float>(ws, L.rec_grad);
  float* gdepth = at<float>(ws, L.grad_depth);
  if (part == 1) {
    {
      PhaseTimer pt(ctx, "raster_backward", s);
      NX_CHECK_HIP(nx::launch_raster_backward(K, at<float4>(ws, L.records), at<uint32_t>(ws, L.inst_ids),
                                              at<uint2>(ws, L.tile_ranges), cd, saved->plain, saved->ids,
                                              saved->weights, saved->tex, saved->n_iter, grad_image, grad_weights,
                                              K > 0 ? gdepth : nullptr, pixel_error, rec_grad, ctx->batch, s));
    }
    PhaseTimer pt(ctx, "preprocess_backward", s);
    NX_CHECK_HIP(nx::launch_preprocess_backward(surfels->means, surfels->quats, surfels->scales, surfels->colors,
                                                ctx->sh, n, cd,
                                                at<uint32_t>(ws, L.tile_counts), rec_grad, grads->means, grads->quats,
                                                grads->scales, grads->opacities, grads->gammas, grads->colors,
                                                pixel_error ? grads->blended_error : nullptr, s));
    return NX_OK;
  }
  {
    PhaseTimer pt(ctx, "zero_record_grads", s);
    NX_CHECK_HIP(nx::launch_fill_f32(rec_grad, 0.0f, (int64_t)nx::kRecGrad * n, s));
  }
  if (K > 0) {
    nx::GridDev gd = make_grid(cam, grid);
    nx::MlpDev md{};
    md.w[0] = mlp->w[0];
    md.w[1] = mlp->w[1];
    md.w[2] = mlp->w[2];
    md.in_dim = mlp->dims[0];
    md.hidden = mlp->dims[1];
    float2* fgrad = grads->table ? at<float2>(ws, L.feat_grad) : nullptr;
    {
      PhaseTimer pt(ctx, "texture_backward", s);
      NX_CHECK_HIP(nx::launch_texture_backward(K, ctx->feat_dtype, ctx->mlp_dtype, ctx->sh, gd, grid->table, md, saved->ids,
                                               saved->depths, saved->weights, grad_image, grad_tex, fgrad,
                                               grads->mlp[0], grads->mlp[1], grads->mlp[2], gdepth,
                                               at<unsigned char>(ws, L.weight_ops), s));
    }
  }
  return NX_OK;
}

// Workspace of nx_render_forward_noalloc: a fixed device array, so that the
// call needs no allocation. Each device that loads the library holds its own
// copy until the process ends. In host code its name is not a device
// address: kernels and copies get the address hipGetSymbolAddress returns
// for the current device, kept per device below.
__device__ __align__(256) unsigned char scratch[NX_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The scratch array's device address on the current device (looked up once
// per device).
int scratch_address(void** out) {
  int dev = -1;
  NX_CHECK_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(NX_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    NX_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(NX_ERR_HIP, "hipGetSymbolAddress returned a null address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return NX_OK;
}

// Turns per-phase timing off for the lifetime of the guard (event creation
// is an allocation the no-allocation entry point must not make).
struct TimingOff {
  nx_ctx* c;
  bool was;
  explicit TimingOff(nx_ctx* ctx) : c(ctx), was(ctx->timing) { c->timing = false; }
  ~TimingOff() { c->timing = was; }
};

}  // namespace

extern "C" {

int nx_version(void) { return 200; }

const char* nx_last_error(void) { return g_last_error.c_str(); }

int nx_create(nx_ctx** out, int32_t K, int32_t tile, nx_dtype feat_dtype, nx_dtype mlp_dtype) {
  if (!out) return fail(NX_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!(K == 0 || K == 1 || K == 2 || K == 4 || K == 8 || K == 16))
    return fail(K < 0 ? NX_ERR_INVALID : NX_ERR_UNSUPPORTED, "K must be one of 0, 1, 2, 4, 8, 16");
  if (tile != 16) return fail(NX_ERR_UNSUPPORTED, "tile must be 16");
  if (feat_dtype != NX_F32 && feat_dtype != NX_F16 && feat_dtype != NX_BF16)
    return fail(NX_ERR_INVALID, "unknown feat_dtype");
  if (mlp_dtype != NX_F32 && mlp_dtype != NX_BF16) return fail(NX_ERR_UNSUPPORTED, "mlp_dtype must be F32 or BF16");
  nx_ctx* c = new nx_ctx();
  c->K = K;
  c->tile = tile;
  c->feat_dtype = feat_dtype;
  c->mlp_dtype = mlp_dtype;
  c->pinned = nullptr;
  c->timing = false;
  hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&c->pinned), sizeof(uint32_t) * 4, hipHostMallocDefault);
  if (e != hipSuccess) {
    delete c;
    return fail(NX_ERR_HIP, std::string("hipHostMalloc: ") + hipGetErrorString(e));
  }
  // set-up of the no-allocation entry point's scratch on the current device
  void* sp = nullptr;
  const int rs = scratch_address(&sp);
  if (rs != NX_OK) {
    (void)hipHostFree(c->pinned);
    delete c;
    return rs;
  }
  *out = c;
  g_last_error.clear();
  return NX_OK;
}

int nx_debug_limits(nx_ctx* ctx, int64_t slab_records, int32_t cas_rounds) {
  int r;
  if ((r = check_ctx(ctx)) != NX_OK) return r;
  if (slab_records < 0 || cas_rounds < 0) return fail(NX_ERR_INVALID, "limits must be >= 0");
  ctx->debug_slab = slab_records;
  ctx->debug_cas = cas_rounds;
  return NX_OK;
}

int nx_set_sh_degree(nx_ctx* ctx, int32_t degree) {
  int r;
  if ((r = check_ctx(ctx)) != NX_OK) return r;
  if (degree != -1 && degree != 3) return fail(NX_ERR_UNSUPPORTED, "sh degree must be -1 (RGB) or 3");
  ctx->sh = degree == 3 ? 1 : 0;
  return NX_OK;
}

int nx_destroy(nx_ctx* ctx) {
  if (!ctx) return NX_OK;
  for (auto& p : ctx->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : ctx->pool) (void)hipEventDestroy(e);
  for (hipEvent_t e : {ctx->ev_fork, ctx->ev_join, ctx->ev_tex, ctx->ev_join2})
    if (e) (void)hipEventDestroy(e);
  for (int a = 0; a < kScatArenas; ++a) {
    if (ctx->ev_bin[a]) (void)hipEventDestroy(ctx->ev_bin[a]);
    if (ctx->ev_red[a]) (void)hipEventDestroy(ctx->ev_red[a]);
  }
  if (ctx->side) (void)hipStreamDestroy(ctx->side);
  if (ctx->side2) (void)hipStreamDestroy(ctx->side2);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  delete ctx;
  return NX_OK;
}

int nx_timing_enable(nx_ctx* ctx, int enabled) {
  int r;
  if ((r = check_ctx(ctx)) != NX_OK) return r;
  ctx->timing = enabled != 0;
  return NX_OK;
}

static int drain_timing(nx_ctx* ctx) {
  for (auto& p : ctx->pending) {
    NX_CHECK_HIP(hipEventSynchronize(p.b));
    float ms = 0.f;
    NX_CHECK_HIP(hipEventElapsedTime(&ms, p.a, p.b));
    ctx->phases[p.phase].ms += ms;
    ctx->phases[p.phase].launches += 1;
    ctx->pool.push_back(p.a);
    ctx->pool.push_back(p.b);
  }
  ctx->pending.clear();
  return NX_OK;
}

int nx_timing_reset(nx_ctx* ctx) {
  int r;
  if ((r = check_ctx(ctx)) != NX_OK) return r;
  if ((r = drain_timing(ctx)) != NX_OK) return r;
  for (auto& p : ctx->phases) {
    p.ms = 0.0;
    p.launches = 0;
  }
  return NX_OK;
}

int nx_timing_get(nx_ctx* ctx, int32_t index, const char** name, double* total_ms, int64_t* launches) {
  int r;
  if ((r = check_ctx(ctx)) != NX_OK) return r;
  if ((r = drain_timing(ctx)) != NX_OK) return r;
  if (index < 0 || index >= (int32_t)ctx->phases.size()) return fail(NX_ERR_INVALID, "timing index out of range");
  if (name) *name = ctx->phases[index].name;
  if (total_ms) *total_ms = ctx->phases[index].ms;
  if (launches) *launches = ctx->phases[index].launches;
  return NX_OK;
}

int nx_workspace_size(nx_ctx* ctx, int64_t n_surfels, const nx_camera* cams, int32_t n_cams, int64_t max_instances,
                      size_t* bytes) {
  int r;
  if ((r = check_ctx(ctx)) != NX_OK) return r;
  if ((r = check_camera(cams, n_cams)) != NX_OK) return r;
  if (!bytes) return fail(NX_ERR_INVALID, "bytes is NULL");
  if (n_surfels < 0 || max_instances < 0) return fail(NX_ERR_INVALID, "negative size");
  size_t total = make_shared_layout(cams, n_cams, ctx->K).total;
  for (int32_t c = 0; c < n_cams; ++c) total += make_layout(n_surfels, make_cam(cams[c]), ctx->K, max_instances).total;
  *bytes = total;
  return NX_OK;
}

int nx_workspace_size_exact(nx_ctx* ctx, const nx_surfels* surfels, const nx_camera* cams, int32_t n_cams,
                            void* workspace, size_t workspace_bytes, size_t* bytes, int64_t* counts, void* stream) {
  int r;
  if ((r = check_ctx(ctx)) != NX_OK) return r;
  if ((r = check_surfels(surfels)) != NX_OK) return r;
  if ((r = check_camera(cams, n_cams)) != NX_OK) return r;
  if (!bytes) return fail(NX_ERR_INVALID, "bytes is NULL");
  size_t need0 = 0;
  for (int32_t c = 0; c < n_cams; ++c) {
    const size_t t = make_layout(surfels->n, make_cam(cams[c]), ctx->K, 0).total;
    need0 = t > need0 ? t : need0;
  }
  if (!workspace || workspace_bytes < need0)
    return fail(NX_ERR_WORKSPACE, "workspace smaller than nx_workspace_size(..., n_cams = 1, max_instances = 0)");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  NX_CHECK_HIP(hipGetLastError());
  size_t total = make_shared_layout(cams, n_cams, ctx->K).total;
  for (int32_t c = 0; c < n_cams; ++c) {
    const nx::CamDev cd = make_cam(cams[c]);
    const Layout L0 = make_layout(surfels->n, cd, ctx->K, 0);
    if ((r = forward_prefix(ctx, surfels, cd, workspace, L0, s)) != NX_OK) return r;
    const uint32_t* offsets = at<uint32_t>(workspace, L0.offsets);
    NX_CHECK_HIP(hipMemcpyAsync(ctx->pinned, offsets + surfels->n, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    NX_CHECK_HIP(hipStreamSynchronize(s));
    const int64_t n_inst = (int64_t)ctx->pinned[0];
    if (counts) counts[c] = n_inst;
    total += make_layout(surfels->n, cd, ctx->K, n_inst).total;
  }
  *bytes = total;
  g_last_error.clear();
  return NX_OK;
}

int nx_workspace_layout(nx_ctx* ctx, int64_t n_surfels, const nx_camera* cams, int32_t n_cams, int64_t n_instances,
                        nx_ws_layout* layout) {
  int r;
  if ((r = check_ctx(ctx)) != NX_OK) return r;
  if ((r = check_camera(cams, n_cams)) != NX_OK) return r;
  if (!layout) return fail(NX_ERR_INVALID, "layout is NULL");
  if (n_cams != 1) return fail(NX_ERR_UNSUPPORTED, "nx_workspace_layout describes one camera");
  if (n_surfels < 0 || n_instances < 0) return fail(NX_ERR_INVALID, "negative size");
  const nx::CamDev cd = make_cam(cams[0]);
  const Layout L = make_layout(n_surfels, cd, ctx->K, n_instances);
  const size_t base = make_shared_layout(cams, n_cams, ctx->K).total;
  layout->depth_keys = base + L.depth_keys;
  layout->tile_counts = base + L.tile_counts;
  layout->rects = base + L.rects;
  layout->records = base + L.records;
  layout->sorted_tiles = base + L.inst_tiles;
  layout->sorted_ids = base + L.inst_ids;
  layout->tile_ranges = base + L.tile_ranges;
  layout->total = base + L.total;
  return NX_OK;
}

int nx_render_forward(nx_ctx* ctx, const nx_surfels* surfels, const nx_camera* cams, int32_t n_cams,
                      const nx_hashgrid* grid, const nx_mlp* mlp, nx_fwd_out* out, void* workspace,
                      size_t workspace_bytes, size_t* workspace_required, void* stream) {
  int r;
  if ((r = check_ctx(ctx)) != NX_OK) return r;
  if ((r = check_surfels(surfels)) != NX_OK) return r;
  if ((r = check_camera(cams, n_cams)) != NX_OK) return r;
  if ((r = check_grid_mlp(ctx, grid, mlp)) != NX_OK) return r;
  if (!out || !out->image || !out->plain || !out->t_final || !out->n_iter || !out->n_instances)
    return fail(NX_ERR_INVALID, "an output pointer is NULL");
  if (ctx->K > 0 && (!out->ids || !out->weights || !out->depths || !out->tex))
    return fail(NX_ERR_INVALID, "an output pointer is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  select_batch(ctx, cams, n_cams);
  NX_CHECK_HIP(hipGetLastError());
  size_t off = make_shared_layout(cams, n_cams, ctx->K).total;
  int64_t pix = 0;
  for (int32_t c = 0; c < n_cams; ++c) {
    const nx_fwd_out oc = camera_slice(ctx, grid, mlp, *out, pix);
    size_t need = 0;
    int64_t n_inst = -1;
    const size_t avail = workspace && workspace_bytes > off ? workspace_bytes - off : 0;
    r = forward_one(ctx, surfels, cams[c], grid, mlp, &oc, workspace ? at<char>(workspace, off) : nullptr, avail,
                    &need, &n_inst, s);
    if (r == NX_ERR_WORKSPACE) {
      // Required size: what is known for cameras <= c, and for the later ones
      // the layout at this camera's instance count (a guess; a second call
      // may ask for more).
      size_t req = off + need;
      const int64_t guess = n_inst > 0 ? n_inst : 0;
      for (int32_t d = c + 1; d < n_cams; ++d) req += make_layout(surfels->n, make_cam(cams[d]), ctx->K, guess).total;
      if (workspace_required) *workspace_required = req;
      if (!workspace_required) return fail(NX_ERR_INVALID, "workspace too small and workspace_required is NULL");
      return fail(NX_ERR_WORKSPACE, "workspace too small");
    }
    if (r != NX_OK) return r;
    out->n_instances[c] = n_inst;
    off += need;
    pix += (int64_t)cams[c].width * cams[c].height;
  }
  if (workspace_required) *workspace_required = off;
  g_last_error.clear();
  return NX_OK;
}

int nx_render_forward_async(nx_ctx* ctx, const nx_surfels* surfels, const nx_camera* cams, int32_t n_cams,
                            const nx_hashgrid* grid, const nx_mlp* mlp, nx_fwd_out* out, int64_t max_instances,
                            void* workspace, size_t workspace_bytes, void* stream) {
  int r;
  if ((r = check_ctx(ctx)) != NX_OK) return r;
  if ((r = check_surfels(surfels)) != NX_OK) return r;
  if ((r = check_camera(cams, n_cams)) != NX_OK) return r;
  if ((r = check_grid_mlp(ctx, grid, mlp)) != NX_OK) return r;
  if (!out || !out->image || !out->plain || !out->t_final || !out->n_iter || !out->n_instances)
    return fail(NX_ERR_INVALID, "an output pointer is NULL");
  if (ctx->K > 0 && (!out->ids || !out->weights || !out->depths || !out->tex))
    return fail(NX_ERR_INVALID, "an output pointer is NULL");
  if (max_instances < 1 || max_instances > 0xFFFFFFFFll)
    return fail(NX_ERR_INVALID, "max_instances must be in [1, 2^32 - 1]");
  const SharedLayout SH = make_shared_layout(cams, n_cams, ctx->K);
  size_t total = SH.total;
  for (int32_t c = 0; c < n_cams; ++c) total += make_layout(surfels->n, make_cam(cams[c]), ctx->K, max_instances).total;
  if (!workspace || workspace_bytes < total)
    return fail(NX_ERR_WORKSPACE, "workspace smaller than nx_workspace_size(..., max_instances)");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  select_batch(ctx, cams, n_cams);
  NX_CHECK_HIP(hipGetLastError());
  size_t off = SH.total;
  int64_t pix = 0;
  for (int32_t c = 0; c < n_cams; ++c) {
    const nx_fwd_out oc = camera_slice(ctx, grid, mlp, *out, pix);
    size_t need = 0;
    int64_t n_inst = -1;
    r = forward_one(ctx, surfels, cams[c], grid, mlp, &oc, at<char>(workspace, off), workspace_bytes - off, &need,
                    &n_inst, s, max_instances);
    if (r != NX_OK) return r;
    out->n_instances[c] = max_instances;
    off += need;
    pix += (int64_t)cams[c].width * cams[c].height;
  }
  g_last_error.clear();
  return NX_OK;
}

int nx_render_forward_noalloc(nx_ctx* ctx, const nx_surfels* surfels, const nx_camera* cams, int32_t n_cams,
                              const nx_hashgrid* grid, const nx_mlp* mlp, nx_fwd_out* out, int64_t max_instances,
                              void* stream) {
  int r;
  if ((r = check_ctx(ctx)) != NX_OK) return r;
  if ((r = check_surfels(surfels)) != NX_OK) return r;
  if ((r = check_camera(cams, n_cams)) != NX_OK) return r;
  if ((r = check_grid_mlp(ctx, grid, mlp)) != NX_OK) return r;
  if (!out || !out->image || !out->plain || !out->t_final || !out->n_iter || !out->n_instances)
    return fail(NX_ERR_INVALID, "an output pointer is NULL");
  if (ctx->K > 0 && (!out->ids || !out->weights || !out->depths || !out->tex))
    return fail(NX_ERR_INVALID, "an output pointer is NULL");
  if (max_instances < 1 || max_instances > 0xFFFFFFFFll)
    return fail(NX_ERR_INVALID, "max_instances must be in [1, 2^32 - 1]");
  size_t total = 0;
  for (int32_t c = 0; c < n_cams; ++c)
    total += make_layout(surfels->n, make_cam(cams[c]), ctx->K, max_instances, true).total;
  if (total > (size_t)NX_NOALLOC_SCRATCH_BYTES)
    return fail(NX_ERR_UNSUPPORTED, "nx_render_forward_noalloc needs " + std::to_string(total) +
                                        " bytes of scratch for these sizes; the library holds " +
                                        std::to_string((size_t)NX_NOALLOC_SCRATCH_BYTES) +
                                        " (use nx_render_forward_async with a workspace)");
  void* ws = nullptr;
  if ((r = scratch_address(&ws)) != NX_OK) return r;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  select_batch(ctx, cams, n_cams);
  NX_CHECK_HIP(hipGetLastError());
  TimingOff no_events(ctx);
  size_t off = 0;
  int64_t pix = 0;
  for (int32_t c = 0; c < n_cams; ++c) {
    const nx_fwd_out oc = camera_slice(ctx, grid, mlp, *out, pix);
    size_t need = 0;
    int64_t n_inst = -1;
    r = forward_one(ctx, surfels, cams[c], grid, mlp, &oc, at<char>(ws, off), (size_t)NX_NOALLOC_SCRATCH_BYTES - off,
                    &need, &n_inst, s, max_instances, true);
    if (r != NX_OK) return r;
    out->n_instances[c] = max_instances;
    off += need;
    pix += (int64_t)cams[c].width * cams[c].height;
  }
  g_last_error.clear();
  return NX_OK;
}

int nx_aux_losses(nx_ctx* ctx, int64_t n_pixels, const float* weights, const float* tex, const float* target,
                  int64_t n_surfels, const float* opacities, const nx_hashgrid* grid, const nx_aux_lambdas* lambdas,
                  float* grad_weights, float* grad_tex, float* grad_opacities, float* grad_table, float* losses,
                  void* stream) {
  int r;
  if ((r = check_ctx(ctx)) != NX_OK) return r;
  if (!lambdas || !losses) return fail(NX_ERR_INVALID, "lambdas or losses is NULL");
  if (n_pixels < 0 || n_surfels < 0) return fail(NX_ERR_INVALID, "negative size");
  if (n_pixels > 0 && ctx->K > 0 && (!weights || !tex || !target))
    return fail(NX_ERR_INVALID, "weights, tex or target is NULL");
  if (n_surfels > 0 && !opacities) return fail(NX_ERR_INVALID, "opacities is NULL");
  for (float v : {lambdas->alpha, lambdas->texture, lambdas->opacity, lambdas->grid})
    if (!isfinite(v)) return fail(NX_ERR_INVALID, "lambdas must be finite");
  if (grid) {
    if (!grid->table || !grid->level_scales) return fail(NX_ERR_INVALID, "grid table or level_scales is NULL");
    if (grid->dtype != ctx->feat_dtype) return fail(NX_ERR_INVALID, "grid dtype differs from the context's feat_dtype");
    if (grid->feat != 2) return fail(NX_ERR_UNSUPPORTED, "only feat == 2 is supported");
    if (grid->levels < 1 || grid->levels > 16) return fail(NX_ERR_UNSUPPORTED, "levels must be in [1, 16]");
    if (grid->log2_size < 4 || grid->log2_size > 24) return fail(NX_ERR_UNSUPPORTED, "log2_size must be in [4, 24]");
    for (int l = 0; l < grid->levels; ++l)
      if (!(grid->level_scales[l] > 0.0f) || !isfinite(grid->level_scales[l]))
        return fail(NX_ERR_INVALID, "level scales must be positive and finite");
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  NX_CHECK_HIP(hipGetLastError());
  NX_CHECK_HIP(nx::launch_aux_losses(n_pixels, ctx->K, weights, tex, target, lambdas->alpha, lambdas->texture,
                                     grad_weights, grad_tex, n_surfels, opacities, lambdas->opacity, grad_opacities,
                                     grid ? grid->dtype : NX_F32, grid ? grid->table : nullptr, grid ? grid->levels : 0,
                                     grid ? grid->log2_size : 0, grid ? grid->level_scales : nullptr, lambdas->grid,
                                     grad_table, losses, s));
  g_last_error.clear();
  return NX_OK;
}

namespace {
constexpr int kFpsMaxGrid = 8192;

struct DensifyLayout {
  size_t keys, ids, tmp_keys, tmp_ids, hist, chosen, keep1, keep2, off1, off2, iota, scan_blocks, total;
};

DensifyLayout densify_layout(int64_t n) {
  DensifyLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  const size_t nn = (size_t)(n > 0 ? n : 1);
  L.keys = take(4 * nn);
  L.ids = take(4 * nn);
  L.tmp_keys = take(4 * nn);
  L.tmp_ids = take(4 * nn);
  L.hist = take(4 * nx::radix_hist_words((int64_t)nn));
  L.chosen = take(4 * nn);
  L.keep1 = take(4 * nn);
  L.keep2 = take(4 * nn);
  L.off1 = take(4 * (nn + 1));
  L.off2 = take(4 * (nn + 1));
  L.iota = take(4 * nn);
  L.scan_blocks = take(4 * nx::scan_block_words((int64_t)nn));
  L.total = o;
  return L;
}

size_t fps_workspace(int64_t n) { return align_up(sizeof(float) * (size_t)(n > 0 ? n : 1)) + nx::fps_slot_bytes(kFpsMaxGrid); }
}  // namespace

int nx_fps_workspace_size(int64_t n, size_t* bytes) {
  if (!bytes || n < 0) return fail(NX_ERR_INVALID, "bad argument");
  *bytes = fps_workspace(n);
  return NX_OK;
}

int nx_fps(nx_ctx* ctx, const float* points, int64_t n, int64_t m, int32_t* order, float* dist2, void* workspace,
           size_t workspace_bytes, void* stream) {
  int r;
  if ((r = check_ctx(ctx)) != NX_OK) return r;
  if (!points || !order || !dist2) return fail(NX_ERR_INVALID, "points, order or dist2 is NULL");
  if (n < 1 || n >= ((int64_t)1 << 31)) return fail(NX_ERR_INVALID, "n must be in [1, 2^31)");
  if (m < 1 || m > n) return fail(NX_ERR_INVALID, "m must be in [1, n]");
  if (!workspace || workspace_bytes < fps_workspace(n)) return fail(NX_ERR_WORKSPACE, "workspace too small");
  int grid = 1;
  NX_CHECK_HIP(nx::fps_grid(n, &grid));
  if (grid > kFpsMaxGrid) grid = kFpsMaxGrid;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  NX_CHECK_HIP(hipGetLastError());
  float* best = static_cast<float*>(workspace);
  void* slots = at<char>(workspace, align_up(sizeof(float) * (size_t)n));
  NX_CHECK_HIP(nx::launch_fps(points, n, m, best, slots, grid, order, dist2, s));
  g_last_error.clear();
  return NX_OK;
}

int nx_densify_workspace_size(int64_t n, size_t* bytes) {
  if (!bytes || n < 0) return fail(NX_ERR_INVALID, "bad argument");
  *bytes = densify_layout(n).total;
  return NX_OK;
}

int nx_densify(nx_ctx* ctx, const nx_surfels* in, const float* blended_error, const float* exp_draws, int64_t n_split,
               float min_opacity, const nx_surfels_out* out, int64_t* n_out, void* workspace, size_t workspace_bytes,
               void* stream) {
  int r;
  if ((r = check_ctx(ctx)) != NX_OK) return r;
  if ((r = check_surfels(in)) != NX_OK) return r;
  const int64_t n = in->n;
  if (!out || !n_out) return fail(NX_ERR_INVALID, "out or n_out is NULL");
  if (n_split < 0) return fail(NX_ERR_INVALID, "n_split is negative");
  if (n_split > n) n_split = n;
  if (n > 0 && (!blended_error || !exp_draws)) return fail(NX_ERR_INVALID, "blended_error or exp_draws is NULL");
  if (!isfinite(min_opacity)) return fail(NX_ERR_INVALID, "min_opacity must be finite");
  if (out->capacity < n + n_split) return fail(NX_ERR_INVALID, "out->capacity is below n + n_split");
  if (n + n_split >= ((int64_t)1 << 31)) return fail(NX_ERR_UNSUPPORTED, "too many surfels");
  if (n + n_split > 0 &&
      (!out->means || !out->quats || !out->scales || !out->opacities || !out->gammas || !out->colors))
    return fail(NX_ERR_INVALID, "an output pointer is NULL");
  const DensifyLayout L = densify_layout(n);
  if (!workspace || workspace_bytes < L.total) return fail(NX_ERR_WORKSPACE, "workspace too small");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  NX_CHECK_HIP(hipGetLastError());
  void* ws = workspace;
  uint32_t* chosen = at<uint32_t>(ws, L.chosen);
  NX_CHECK_HIP(nx::launch_split_select(n, n_split, blended_error, exp_draws, at<uint32_t>(ws, L.keys),
                                       at<uint32_t>(ws, L.ids), at<uint32_t>(ws, L.tmp_keys),
                                       at<uint32_t>(ws, L.tmp_ids), at<uint32_t>(ws, L.hist), chosen, s));
  uint32_t* off1 = at<uint32_t>(ws, L.off1);
  uint32_t* off2 = at<uint32_t>(ws, L.off2);
  NX_CHECK_HIP(nx::launch_split_prune(n, in->means, in->quats, in->scales, in->opacities, in->gammas, in->colors,
                                      chosen, min_opacity, at<uint32_t>(ws, L.keep1), at<uint32_t>(ws, L.keep2), off1,
                                      off2, at<uint32_t>(ws, L.iota), at<uint32_t>(ws, L.scan_blocks), out->means,
                                      out->quats, out->scales, out->opacities, out->gammas, out->colors, out->parent,
                                      s));
  NX_CHECK_HIP(hipMemcpyAsync(ctx->pinned, off1 + n, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  NX_CHECK_HIP(hipMemcpyAsync(ctx->pinned + 1, off2 + n, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  NX_CHECK_HIP(hipStreamSynchronize(s));
  *n_out = (int64_t)ctx->pinned[0] + (int64_t)ctx->pinned[1];
  g_last_error.clear();
  return NX_OK;
}

int nx_instance_counts(nx_ctx* ctx, int64_t n_surfels, const nx_camera* cams, int32_t n_cams,
                       const int64_t* n_instances, const void* workspace, size_t workspace_bytes, int64_t* counts,
                       void* stream) {
  int r;
  if ((r = check_ctx(ctx)) != NX_OK) return r;
  if ((r = check_camera(cams, n_cams)) != NX_OK) return r;
  if (n_surfels < 0 || !n_instances || !counts) return fail(NX_ERR_INVALID, "bad argument");
  size_t off = make_shared_layout(cams, n_cams, ctx->K).total;
  for (int32_t c = 0; c < n_cams; ++c) {
    if (n_instances[c] < 0) return fail(NX_ERR_INVALID, "n_instances is negative");
    off += make_layout(n_surfels, make_cam(cams[c]), ctx->K, n_instances[c]).total;
  }
  if (!workspace || workspace_bytes < off) return fail(NX_ERR_INVALID, "workspace does not match the forward");
  NX_CHECK_HIP(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)));
  off = make_shared_layout(cams, n_cams, ctx->K).total;
  for (int32_t c = 0; c < n_cams; ++c) {
    const Layout L = make_layout(n_surfels, make_cam(cams[c]), ctx->K, n_instances[c]);
    uint32_t v = 0;
    NX_CHECK_HIP(hipMemcpy(&v, at<char>(workspace, off + L.offsets + sizeof(uint32_t) * (size_t)n_surfels),
                           sizeof(uint32_t), hipMemcpyDeviceToHost));
    counts[c] = (int64_t)v;
    off += L.total;
  }
  g_last_error.clear();
  return NX_OK;
}

int nx_autotune_raster(nx_ctx* ctx, const nx_surfels* surfels, const nx_camera* cams, int32_t n_cams,
                       const nx_fwd_out* out, const void* workspace, size_t workspace_bytes, int32_t reps,
                       int32_t* batch, void* stream) {
  int r;
  if ((r = check_ctx(ctx)) != NX_OK) return r;
  if ((r = check_surfels(surfels)) != NX_OK) return r;
  if ((r = check_camera(cams, n_cams)) != NX_OK) return r;
  if (!out || !out->plain || !out->t_final || !out->n_iter || !out->n_instances)
    return fail(NX_ERR_INVALID, "an output pointer is NULL");
  if (ctx->K > 0 && (!out->ids || !out->weights || !out->depths))
    return fail(NX_ERR_INVALID, "an output pointer is NULL");
  if (reps < 1 || reps > 100) return fail(NX_ERR_INVALID, "reps must be in [1, 100]");
  if (!batch) return fail(NX_ERR_INVALID, "batch is NULL");
  size_t total = make_shared_layout(cams, n_cams, ctx->K).total;
  for (int32_t c = 0; c < n_cams; ++c) {
    if (out->n_instances[c] < 0) return fail(NX_ERR_INVALID, "n_instances is negative");
    total += make_layout(surfels->n, make_cam(cams[c]), ctx->K, out->n_instances[c]).total;
  }
  if (!workspace || workspace_bytes < total) return fail(NX_ERR_INVALID, "workspace does not match the forward");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  NX_CHECK_HIP(hipGetLastError());
  struct Events {
    hipEvent_t e[2] = {nullptr, nullptr};
    ~Events() {
      for (hipEvent_t x : e)
        if (x) (void)hipEventDestroy(x);
    }
  } ev;
  NX_CHECK_HIP(hipEventCreate(&ev.e[0]));
  NX_CHECK_HIP(hipEventCreate(&ev.e[1]));
  const int64_t K = ctx->K;
  // the collection pass of every camera with LDS batch b
  auto run = [&](int b) -> hipError_t {
    size_t off = make_shared_layout(cams, n_cams, ctx->K).total;
    int64_t pix = 0;
    for (int32_t c = 0; c < n_cams; ++c) {
      const nx::CamDev cd = make_cam(cams[c]);
      const Layout L = make_layout(surfels->n, cd, ctx->K, out->n_instances[c]);
      char* ws = const_cast<char*>(static_cast<const char*>(workspace)) + off;
      const hipError_t e = nx::launch_raster_forward(
          ctx->K, at<float4>(ws, L.records), at<uint32_t>(ws, L.inst_ids), at<uint2>(ws, L.tile_ranges), cd,
          out->plain + 3 * pix, K > 0 ? out->ids + K * pix : nullptr, K > 0 ? out->weights + K * pix : nullptr,
          K > 0 ? out->depths + K * pix : nullptr, out->t_final + pix, out->n_iter + pix, b, s);
      if (e != hipSuccess) return e;
      off += L.total;
      pix += (int64_t)cams[c].width * cams[c].height;
    }
    return hipSuccess;
  };
  int best_b = nx::kRasterBatchDefault;
  float best_ms = 0.0f;
  for (int b : nx::kRasterBatches) {
    NX_CHECK_HIP(run(b));  // warm-up
    NX_CHECK_HIP(hipEventRecord(ev.e[0], s));
    for (int32_t k = 0; k < reps; ++k) NX_CHECK_HIP(run(b));
    NX_CHECK_HIP(hipEventRecord(ev.e[1], s));
    NX_CHECK_HIP(hipEventSynchronize(ev.e[1]));
    float ms = 0.0f;
    NX_CHECK_HIP(hipEventElapsedTime(&ms, ev.e[0], ev.e[1]));
    if (b == nx::kRasterBatches[0] || ms < best_ms) {
      best_ms = ms;
      best_b = b;
    }
  }
  ctx->tuned_batch[camera_key(ctx->K, cams, n_cams)] = best_b;
  *batch = best_b;
  g_last_error.clear();
  return NX_OK;
}

int nx_render_backward(nx_ctx* ctx, const nx_surfels* surfels, const nx_camera* cams, int32_t n_cams,
                       const nx_hashgrid* grid, const nx_mlp* mlp, const nx_fwd_out* saved, const void* workspace,
                       size_t workspace_bytes, const float* grad_image, const float* grad_weights,
                       const float* grad_tex, const nx_grads* grads, void* stream) {
  int r;
  if ((r = check_ctx(ctx)) != NX_OK) return r;
  if ((r = check_surfels(surfels)) != NX_OK) return r;
  if ((r = check_camera(cams, n_cams)) != NX_OK) return r;
  if ((r = check_grid_mlp(ctx, grid, mlp)) != NX_OK) return r;
  if (!saved || !saved->plain || !saved->n_iter || !saved->n_instances)
    return fail(NX_ERR_INVALID, "saved forward outputs are NULL");
  if (ctx->K > 0 && (!saved->ids || !saved->weights || !saved->depths || !saved->tex))
    return fail(NX_ERR_INVALID, "saved forward outputs are NULL");
  if (!grad_image) return fail(NX_ERR_INVALID, "grad_image is NULL");
  if (!grads) return fail(NX_ERR_INVALID, "grads is NULL");
  const SharedLayout SH = make_shared_layout(cams, n_cams, ctx->K);
  if (SH.capacity >= (1ll << 32))
    return fail(NX_ERR_UNSUPPORTED, "too many samples (pixels x K) in one call for the hash-grid backward (limit about 4e8)");
  size_t total = SH.total;
  for (int32_t c = 0; c < n_cams; ++c) {
    if (saved->n_instances[c] < 0) return fail(NX_ERR_INVALID, "saved n_instances is negative");
    total += make_layout(surfels->n, make_cam(cams[c]), ctx->K, saved->n_instances[c]).total;
  }
  if (!workspace || workspace_bytes < total) return fail(NX_ERR_INVALID, "workspace does not match the forward");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  select_batch(ctx, cams, n_cams);
  NX_CHECK_HIP(hipGetLastError());
  void* ws = const_cast<void*>(workspace);
  const int64_t K = ctx->K > 0 ? ctx->K : 0;
  // 1. per camera: texture backward (writes its per-level feature
  //    gradients), collection-pass backward, preprocess backward
  if ((r = side_streams(ctx)) != NX_OK) return r;
  // texture backward of every camera on the call's stream; then the
  // collection-pass and preprocess backward of every camera on side2, which
  // overlap the hash-grid gradient below (they would only take CUs from the
  // next camera's texture backward if they started earlier)
  for (int part = 0; part < 2; ++part) {
    hipStream_t sp = part == 0 ? s : ctx->side2;
    if (part == 1) {
      NX_CHECK_HIP(hipEventRecord(ctx->ev_tex, s));
      NX_CHECK_HIP(hipStreamWaitEvent(ctx->side2, ctx->ev_tex, 0));
    }
    size_t off = SH.total;
    int64_t pix = 0;
    for (int32_t c = 0; c < n_cams; ++c) {
      const nx_fwd_out sc = camera_slice(ctx, grid, mlp, *saved, pix);
      const int64_t n_inst = saved->n_instances[c];
      r = backward_one(ctx, surfels, cams[c], grid, mlp, &sc, n_inst, at<char>(ws, off), grad_image + 3 * pix,
                       grad_weights ? grad_weights + K * pix : nullptr, grad_tex ? grad_tex + 3 * K * pix : nullptr,
                       grads, (grads->pixel_error && grads->blended_error) ? grads->pixel_error + pix : nullptr, sp,
                       part);
      if (r != NX_OK) return r;
      off += make_layout(surfels->n, make_cam(cams[c]), ctx->K, n_inst).total;
      pix += (int64_t)cams[c].width * cams[c].height;
    }
  }
  // 2. hash-grid gradient, level by level: one joint bin launch files the
  //    records of every camera, then one reduction per level
  if (K > 0 && grads->table && SH.blocks > 0) {
    const nx::GridDev gd0 = make_grid(cams[0], grid);
    nx::ScatterCam* dcams = at<nx::ScatterCam>(ws, SH.cams);
    nx::ScatterCam cam0{};
    {
      size_t coff = SH.total;
      int64_t cpix = 0, blk0 = 0;
      for (int32_t c = 0; c < n_cams; ++c) {
        const nx::CamDev cd = make_cam(cams[c]);
        const Layout L = make_layout(surfels->n, cd, ctx->K, saved->n_instances[c]);
        const nx::ScatterGeom sg = nx::scatter_geom(cams[c].width, cams[c].height, ctx->K);
        nx::ScatterCam sc;
        sc.gd = make_grid(cams[c], grid);
        sc.depths = saved->depths + K * cpix;
        sc.feat_grad = at<float2>(ws, coff + L.feat_grad);
        sc.bw = sg.bw;
        sc.bh = sg.bh;
        sc.nbx = sg.nbx;
        sc.nby = sg.nby;
        sc.blk0 = blk0;
        if (c == 0) cam0 = sc;
        if (n_cams > 1) NX_CHECK_HIP(nx::launch_write_scatter_cam(sc, dcams + c, s));
        blk0 += (int64_t)sg.nbx * sg.nby;
        coff += L.total;
        cpix += (int64_t)cams[c].width * cams[c].height;
      }
    }
    // Level l: bin on the call's stream into arena l % kScatArenas, reduce on
    // the side stream; the bin of level l + kScatArenas waits for the reduce
    // of level l (same arena), the reduce of level l for its own bin; the
    // call's stream waits for the last reduce at the end.
    NX_CHECK_HIP(hipEventRecord(ctx->ev_fork, s));
    NX_CHECK_HIP(hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0));
    for (int l = 0; l < gd0.levels; ++l) {
      const int a = l % kScatArenas;
      uint16_t* rk = at<uint16_t>(ws, SH.rec_key[a]);
      float2* rv = at<float2>(ws, SH.rec_val[a]);
      uint2* tab = at<uint2>(ws, SH.slab_table[a]);
      if (l >= kScatArenas) NX_CHECK_HIP(hipStreamWaitEvent(s, ctx->ev_red[a], 0));
      {
        PhaseTimer pt(ctx, "scatter_bin", s);
        NX_CHECK_HIP(nx::launch_hash_scatter_bin(ctx->K, cam0, dcams, n_cams, SH.blocks, gd0, l, grads->table,
                                                 SH.rows, tab, rk, rv, ctx->debug_slab, s));
      }
      NX_CHECK_HIP(hipEventRecord(ctx->ev_bin[a], s));
      NX_CHECK_HIP(hipStreamWaitEvent(ctx->side, ctx->ev_bin[a], 0));
      {
        PhaseTimer pt(ctx, "scatter_reduce", ctx->side);
        NX_CHECK_HIP(nx::launch_hash_scatter_reduce(gd0, l, grads->table, SH.rows, SH.blocks, tab, rk, rv, ctx->debug_cas,
                                                    ctx->side));
      }
      NX_CHECK_HIP(hipEventRecord(ctx->ev_red[a], ctx->side));
    }
    NX_CHECK_HIP(hipEventRecord(ctx->ev_join, ctx->side));
    NX_CHECK_HIP(hipStreamWaitEvent(s, ctx->ev_join, 0));
  }
  NX_CHECK_HIP(hipEventRecord(ctx->ev_join2, ctx->side2));
  NX_CHECK_HIP(hipStreamWaitEvent(s, ctx->ev_join2, 0));
  g_last_error.clear();
  return NX_OK;
}

}  // extern "C"
