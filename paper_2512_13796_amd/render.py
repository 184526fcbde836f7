"""Python binding of the rendering library: argument marshalling only.

Every step of the rendering path runs in the HIP kernels of libnexels.so;
this module allocates output and workspace tensors with PyTorch, fills the
C structs of include/nexels.h and calls nx_render_forward /
nx_render_backward on the current HIP stream. ``RenderFunction`` wraps the
two calls as a torch.autograd.Function.
"""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np
import torch

from . import _lib as L

_DTYPE = {torch.float32: L.NX_F32, torch.float16: L.NX_F16, torch.bfloat16: L.NX_BF16}


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check_dev(name, t, device, dtype=None, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a tensor")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def camera_struct(cam, near=0.2):
    """nx_camera from an object with world_to_cam [3,4], fx, fy, cx, cy, width, height."""
    c = L.NxCamera()
    m = np.asarray(cam.world_to_cam, dtype=np.float64).reshape(-1)
    for i in range(12):
        c.world_to_cam[i] = float(m[i])
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.near_z = float(near)
    c.width, c.height = int(cam.width), int(cam.height)
    return c


class Context:
    """Owns one nx_ctx (K, tile size, storage dtypes, appearance).

    sh_degree=3 selects the spherical-harmonics appearance: surfel colours are
    [n, 48] coefficients ([16][3]) and the MLP head has 48 outputs; None keeps
    RGB colours and a sigmoid head of 3."""

    def __init__(self, K, feat_dtype=torch.float32, mlp_dtype=torch.float32, sh_degree=None):
        self.lib = L.load()
        self.K = int(K)
        self.feat_dtype = feat_dtype
        self.mlp_dtype = mlp_dtype
        self.sh_degree = sh_degree
        h = ctypes.c_void_p()
        L.check(self.lib.nx_create(ctypes.byref(h), self.K, 16, _DTYPE[feat_dtype], _DTYPE[mlp_dtype]))
        self.handle = h
        if sh_degree is not None:
            L.check(self.lib.nx_set_sh_degree(h, int(sh_degree)))
        self.ws_hint = 0

    def debug_limits(self, slab_records=0, cas_rounds=0):
        """nx_debug_limits: force the hash-grid gradient's slab-overflow and lost-CAS fallbacks (0 = default)."""
        L.check(self.lib.nx_debug_limits(self.handle, int(slab_records), int(cas_rounds)))

    @property
    def n_color(self):
        return 3 if self.sh_degree is None else 3 * (self.sh_degree + 1) ** 2

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            self.lib.nx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def timing(self, enabled=True):
        L.check(self.lib.nx_timing_enable(self.handle, 1 if enabled else 0))

    def timing_reset(self):
        L.check(self.lib.nx_timing_reset(self.handle))

    def timings(self):
        """{phase: (total_ms, launches)} accumulated since the last reset."""
        out = {}
        i = 0
        while True:
            nm = ctypes.c_char_p()
            ms = ctypes.c_double()
            cnt = ctypes.c_int64()
            if self.lib.nx_timing_get(self.handle, i, ctypes.byref(nm), ctypes.byref(ms), ctypes.byref(cnt)) != 0:
                break
            out[nm.value.decode()] = (ms.value, cnt.value)
            i += 1
        return out

    def workspace_layout(self, n_surfels, cam, n_instances, near=0.2):
        lay = L.NxWsLayout()
        cs = camera_struct(cam, near)
        L.check(self.lib.nx_workspace_layout(self.handle, int(n_surfels), ctypes.byref(cs), 1, int(n_instances),
                                             ctypes.byref(lay)))
        return {f: getattr(lay, f) for f, _ in L.NxWsLayout._fields_}


@dataclasses.dataclass
class ForwardResult:
    image: torch.Tensor
    plain: torch.Tensor
    ids: torch.Tensor
    weights: torch.Tensor
    depths: torch.Tensor
    t_final: torch.Tensor
    tex: torch.Tensor
    n_iter: torch.Tensor
    n_instances: int  # total over the cameras
    workspace: torch.Tensor
    camera: object = None  # the camera, or the list of cameras, the call rendered
    n_instances_cam: list = None
    near: float = 0.2
    cells: torch.Tensor = None
    relu_masks: torch.Tensor = None
    features: torch.Tensor = None


def _surfel_struct(ctx, surfels, device):
    means, quats, scales, opac, gammas, colors = surfels
    n = means.shape[0]
    for nm, t, shp in (("means", means, (n, 3)), ("quats", quats, (n, 4)), ("scales", scales, (n, 2)),
                       ("opacities", opac, (n,)), ("gammas", gammas, (n, 2)), ("colors", colors, (n, ctx.n_color))):
        _check_dev(nm, t, device, torch.float32, shp)
    return L.NxSurfels(_ptr(means), _ptr(quats), _ptr(scales), _ptr(opac), _ptr(gammas), _ptr(colors), n)


def _structs(ctx, surfels, table, level_scales, weights, device):
    s = _surfel_struct(ctx, surfels, device)
    g = L.NxHashGrid()
    m = L.NxMLP()
    keep = []
    if ctx.K > 0:
        _check_dev("table", table, device, ctx.feat_dtype)
        ls = level_scales.detach().to("cpu", torch.float32).contiguous()
        keep.append(ls)
        g.table = _ptr(table)
        g.dtype = _DTYPE[table.dtype]
        g.levels, g.log2_size, g.feat = table.shape[0], int(table.shape[1]).bit_length() - 1, table.shape[2]
        if (1 << g.log2_size) != table.shape[1]:
            raise ValueError("table size must be a power of two")
        g.level_scales = ctypes.c_void_p(ls.data_ptr())
        for i, w in enumerate(weights):
            _check_dev(f"mlp[{i}]", w, device, ctx.mlp_dtype)
            m.w[i] = w.data_ptr()
        m.dtype = _DTYPE[ctx.mlp_dtype]
        m.dims[0] = weights[0].shape[1]
        m.dims[1] = weights[0].shape[0]
        m.dims[2] = weights[1].shape[0]
        m.dims[3] = weights[2].shape[0]
    return s, g, m, keep


def _cameras(cam):
    return list(cam) if isinstance(cam, (list, tuple)) else [cam]


def workspace_size(ctx: Context, n_surfels, cam, max_instances, near=0.2):
    """nx_workspace_size for one camera or a list of cameras."""
    cams = _cameras(cam)
    cs = (L.NxCamera * len(cams))(*[camera_struct(c, near) for c in cams])
    size = ctypes.c_size_t()
    L.check(ctx.lib.nx_workspace_size(ctx.handle, int(n_surfels), cs, len(cams), int(max_instances),
                                      ctypes.byref(size)))
    return int(size.value)


def workspace_size_exact(ctx: Context, surfels, cam, near=0.2):
    """nx_workspace_size_exact: (bytes nx_render_forward needs, per-camera pair counts) for these surfels and
    cameras (one synchronisation per camera)."""
    device = surfels[0].device
    s = _surfel_struct(ctx, surfels, device)
    cams = _cameras(cam)
    cs = (L.NxCamera * len(cams))(*[camera_struct(c, near) for c in cams])
    need = max(workspace_size(ctx, surfels[0].shape[0], c, 0, near) for c in cams)
    ws = torch.empty(need, device=device, dtype=torch.uint8)
    size = ctypes.c_size_t()
    counts = (ctypes.c_int64 * len(cams))()
    stream = ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)
    L.check(ctx.lib.nx_workspace_size_exact(ctx.handle, ctypes.byref(s), cs, len(cams), _ptr(ws), ws.numel(),
                                            ctypes.byref(size), counts, stream))
    return int(size.value), [int(v) for v in counts]


def instance_counts(ctx: Context, n_surfels, res: ForwardResult):
    """True (surfel, tile) pair counts per camera of the forward that produced res (nx_instance_counts;
    synchronises the current stream)."""
    cams = _cameras(res.camera)
    cs = (L.NxCamera * len(cams))(*[camera_struct(c, res.near) for c in cams])
    lay = (ctypes.c_int64 * len(cams))(*res.n_instances_cam)
    out = (ctypes.c_int64 * len(cams))()
    stream = ctypes.c_void_p(torch.cuda.current_stream(res.workspace.device).cuda_stream)
    L.check(ctx.lib.nx_instance_counts(ctx.handle, int(n_surfels), cs, len(cams), lay, _ptr(res.workspace),
                                       res.workspace.numel(), out, stream))
    return [int(v) for v in out]


def autotune_raster(ctx: Context, surfels, res: ForwardResult, reps=5):
    """nx_autotune_raster: choose the collection pass's LDS batch for the cameras of res (the result of a
    finished forward with these surfels), keep it in ctx for later calls over cameras of the same sizes, and
    return it. Synchronises the current stream."""
    device = surfels[0].device
    s = _surfel_struct(ctx, surfels, device)
    cams = _cameras(res.camera)
    cs = (L.NxCamera * len(cams))(*[camera_struct(c, res.near) for c in cams])
    n_inst = (ctypes.c_int64 * len(cams))(*res.n_instances_cam)
    out = L.NxFwdOut(_ptr(res.image), _ptr(res.plain), _ptr(res.ids), _ptr(res.weights), _ptr(res.depths),
                     _ptr(res.t_final), _ptr(res.tex), _ptr(res.n_iter), None, None, None, n_inst)
    batch = ctypes.c_int32()
    stream = ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)
    L.check(ctx.lib.nx_autotune_raster(ctx.handle, ctypes.byref(s), cs, len(cams), ctypes.byref(out),
                                       _ptr(res.workspace), res.workspace.numel(), int(reps), ctypes.byref(batch),
                                       stream))
    return int(batch.value)


def render_forward(ctx: Context, surfels, cam, table=None, level_scales=None, weights=None, near=0.2,
                   workspace=None, want_cells=False, max_instances=None) -> ForwardResult:
    """Collection and texturing passes (nx_render_forward) for one camera or a
    list of cameras; with several cameras every per-pixel output holds the
    cameras one after another.

    max_instances (per camera) selects nx_render_forward_async: no host
    synchronisation, the workspace laid out for that many (surfel, tile)
    pairs (allocated here unless `workspace` is given), n_instances_cam set
    to that bound and n_instances to -1; instance_counts() reads the true
    counts.

    want_cells=True also returns the hash-grid lattice cells the texturing
    pass used ([P, K, levels, 3] int32), its ReLU decisions
    ([P, K, 2*hidden/32] int32 bit masks) and the MLP inputs it formed
    ([P, K, levels*feat] float32), for decision-level comparisons."""
    device = surfels[0].device
    s, g, m, keep = _structs(ctx, surfels, table, level_scales, weights, device)
    cams = _cameras(cam)
    cs = (L.NxCamera * len(cams))(*[camera_struct(c, near) for c in cams])
    P = sum(c.width * c.height for c in cams)
    K = ctx.K
    f32 = dict(device=device, dtype=torch.float32)
    res = ForwardResult(
        image=torch.empty(P, 3, **f32), plain=torch.empty(P, 3, **f32),
        ids=torch.empty(P, max(K, 1), device=device, dtype=torch.int32),
        weights=torch.empty(P, max(K, 1), **f32), depths=torch.empty(P, max(K, 1), **f32),
        t_final=torch.empty(P, **f32), tex=torch.empty(P, max(K, 1), 3, **f32),
        n_iter=torch.empty(P, device=device, dtype=torch.int32), n_instances=0, workspace=None, camera=cam,
        near=near)
    if want_cells and K > 0:
        res.cells = torch.zeros(P, K, table.shape[0], 3, device=device, dtype=torch.int32)
        res.relu_masks = torch.zeros(P, K, 2 * weights[0].shape[0] // 32, device=device, dtype=torch.int32)
        res.features = torch.zeros(P, K, table.shape[0] * table.shape[2], device=device, dtype=torch.float32)
    n_inst = (ctypes.c_int64 * len(cams))()
    out = L.NxFwdOut(_ptr(res.image), _ptr(res.plain), _ptr(res.ids), _ptr(res.weights), _ptr(res.depths),
                     _ptr(res.t_final), _ptr(res.tex), _ptr(res.n_iter), _ptr(res.cells), _ptr(res.relu_masks),
                     _ptr(res.features), n_inst)
    stream = ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)
    if max_instances is not None:
        size = workspace_size(ctx, surfels[0].shape[0], cams, max_instances, near)
        ws = workspace if workspace is not None else torch.empty(size, device=device, dtype=torch.uint8)
        L.check(ctx.lib.nx_render_forward_async(ctx.handle, ctypes.byref(s), cs, len(cams), ctypes.byref(g),
                                                ctypes.byref(m), ctypes.byref(out), int(max_instances), _ptr(ws),
                                                ws.numel(), stream))
        res.n_instances_cam = [int(v) for v in n_inst]
        res.n_instances = -1
        res.workspace = ws
        del keep
        return res
    need = ctypes.c_size_t(0)
    ws = workspace
    for _ in range(len(cams) + 3):
        if ws is None or ws.numel() < ctx.ws_hint:
            ws = torch.empty(max(ctx.ws_hint, 256), device=device, dtype=torch.uint8)
        code = ctx.lib.nx_render_forward(ctx.handle, ctypes.byref(s), cs, len(cams), ctypes.byref(g),
                                         ctypes.byref(m), ctypes.byref(out), _ptr(ws), ws.numel(),
                                         ctypes.byref(need), stream)
        if code == L.NX_ERR_WORKSPACE:
            ctx.ws_hint = max(ctx.ws_hint, int(need.value))
            ws = None
            continue
        L.check(code)
        break
    else:
        raise L.NexelsError(L.NX_ERR_WORKSPACE, "workspace sizing did not converge")
    ctx.ws_hint = max(ctx.ws_hint, int(need.value))
    res.n_instances_cam = [int(v) for v in n_inst]
    res.n_instances = sum(res.n_instances_cam)
    res.workspace = ws
    del keep
    return res


def render_forward_noalloc(ctx: Context, surfels, cam, table=None, level_scales=None, weights=None,
                           max_instances=1, near=0.2) -> ForwardResult:
    """nx_render_forward_noalloc: the forward without a workspace argument (the
    library's fixed scratch array holds the intermediates; nothing is
    allocated inside the call and the host does not wait). The output tensors
    are allocated here, before the call. The result has no workspace, so it
    cannot feed render_backward."""
    device = surfels[0].device
    s, g, m, keep = _structs(ctx, surfels, table, level_scales, weights, device)
    cams = _cameras(cam)
    cs = (L.NxCamera * len(cams))(*[camera_struct(c, near) for c in cams])
    P = sum(c.width * c.height for c in cams)
    K = ctx.K
    f32 = dict(device=device, dtype=torch.float32)
    res = ForwardResult(
        image=torch.empty(P, 3, **f32), plain=torch.empty(P, 3, **f32),
        ids=torch.empty(P, max(K, 1), device=device, dtype=torch.int32),
        weights=torch.empty(P, max(K, 1), **f32), depths=torch.empty(P, max(K, 1), **f32),
        t_final=torch.empty(P, **f32), tex=torch.empty(P, max(K, 1), 3, **f32),
        n_iter=torch.empty(P, device=device, dtype=torch.int32), n_instances=-1, workspace=None, camera=cam,
        near=near)
    n_inst = (ctypes.c_int64 * len(cams))()
    out = L.NxFwdOut(_ptr(res.image), _ptr(res.plain), _ptr(res.ids), _ptr(res.weights), _ptr(res.depths),
                     _ptr(res.t_final), _ptr(res.tex), _ptr(res.n_iter), None, None, None, n_inst)
    stream = ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)
    L.check(ctx.lib.nx_render_forward_noalloc(ctx.handle, ctypes.byref(s), cs, len(cams), ctypes.byref(g),
                                              ctypes.byref(m), ctypes.byref(out), int(max_instances), stream))
    res.n_instances_cam = [int(v) for v in n_inst]
    del keep
    return res


def render_backward(ctx: Context, surfels, fwd: ForwardResult, table=None, level_scales=None, weights=None,
                    grad_image=None, grad_weights=None, grad_tex=None, grads=None, pixel_error=None):
    """Accumulate gradients into ``grads`` (dict of float32 tensors; missing keys are skipped).

    pixel_error [P] (optional) adds the blended errors sum_p w_{i,p} pixel_error[p] into grads["blended_error"]
    [n] (the densification signal)."""
    device = surfels[0].device
    s, g, m, keep = _structs(ctx, surfels, table, level_scales, weights, device)
    cams = _cameras(fwd.camera)
    cs = (L.NxCamera * len(cams))(*[camera_struct(c, fwd.near) for c in cams])
    P = sum(c.width * c.height for c in cams)
    K = ctx.K
    _check_dev("grad_image", grad_image, device, torch.float32, (P, 3))
    if grad_weights is not None:
        _check_dev("grad_weights", grad_weights, device, torch.float32, (P, K))
    if grad_tex is not None:
        _check_dev("grad_tex", grad_tex, device, torch.float32, (P, K, 3))
    grads = grads or {}
    for k, t in grads.items():
        if t is not None and k != "mlp":
            _check_dev(f"grads[{k}]", t, device, torch.float32)
    gm = grads.get("mlp") or [None, None, None]
    gs = L.NxGrads(_ptr(grads.get("means")), _ptr(grads.get("quats")), _ptr(grads.get("scales")),
                   _ptr(grads.get("opacities")), _ptr(grads.get("gammas")), _ptr(grads.get("colors")),
                   _ptr(grads.get("table")))
    for i in range(3):
        gs.mlp[i] = None if gm[i] is None else gm[i].data_ptr()
    if pixel_error is not None:
        _check_dev("pixel_error", pixel_error, device, torch.float32, (P,))
        _check_dev("grads[blended_error]", grads["blended_error"], device, torch.float32, (surfels[0].shape[0],))
        gs.pixel_error = _ptr(pixel_error)
        gs.blended_error = _ptr(grads["blended_error"])
    n_inst = (ctypes.c_int64 * len(cams))(*fwd.n_instances_cam)
    out = L.NxFwdOut(_ptr(fwd.image), _ptr(fwd.plain), _ptr(fwd.ids), _ptr(fwd.weights), _ptr(fwd.depths),
                     _ptr(fwd.t_final), _ptr(fwd.tex), _ptr(fwd.n_iter), None, None, None, n_inst)
    stream = ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)
    L.check(ctx.lib.nx_render_backward(ctx.handle, ctypes.byref(s), cs, len(cams), ctypes.byref(g),
                                       ctypes.byref(m), ctypes.byref(out), _ptr(fwd.workspace), fwd.workspace.numel(),
                                       _ptr(grad_image), _ptr(grad_weights), _ptr(grad_tex), ctypes.byref(gs),
                                       stream))
    del keep
    return grads


def aux_losses(ctx: Context, weights, tex, target, opacities, table=None, level_scales=None,
               lambdas=(1.0, 1.0, 1.0, 1.0), grads=None):
    """nx_aux_losses: the losses L_alpha, L_texture, L_opacity, L_grid (unweighted, a float32 [4] device
    tensor) of a forward's weights [P,K] and tex [P,K,3] against target [P,3], of the opacities [n] and of the
    table (optional); the gradient of their lambda-weighted sum is added to the float32 tensors in ``grads``
    (keys "weights", "tex", "opacities", "table"; missing keys are skipped)."""
    device = opacities.device
    P = target.shape[0]
    K = ctx.K
    _check_dev("target", target, device, torch.float32, (P, 3))
    _check_dev("opacities", opacities, device, torch.float32)
    if K > 0:
        _check_dev("weights", weights, device, torch.float32, (P, K))
        _check_dev("tex", tex, device, torch.float32, (P, K, 3))
    grads = grads or {}
    for k, t in grads.items():
        _check_dev(f"grads[{k}]", t, device, torch.float32)
    g = None
    keep = []
    if table is not None:
        _check_dev("table", table, device, ctx.feat_dtype)
        ls = level_scales.detach().to("cpu", torch.float32).contiguous()
        keep.append(ls)
        g = L.NxHashGrid()
        g.table = _ptr(table)
        g.dtype = _DTYPE[table.dtype]
        g.levels, g.log2_size, g.feat = table.shape[0], int(table.shape[1]).bit_length() - 1, table.shape[2]
        g.level_scales = ctypes.c_void_p(ls.data_ptr())
    lam = L.NxAuxLambdas(*[float(v) for v in lambdas])
    losses = torch.empty(4, device=device, dtype=torch.float32)
    stream = ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)
    L.check(ctx.lib.nx_aux_losses(ctx.handle, P, _ptr(weights if K > 0 else None), _ptr(tex if K > 0 else None),
                                  _ptr(target), opacities.shape[0], _ptr(opacities),
                                  None if g is None else ctypes.byref(g), ctypes.byref(lam),
                                  _ptr(grads.get("weights")), _ptr(grads.get("tex")), _ptr(grads.get("opacities")),
                                  _ptr(grads.get("table")), _ptr(losses), stream))
    del keep
    return losses


def fps(ctx: Context, points, m):
    """nx_fps: the first m points of the farthest-point-sampling order of points [n,3] (device float32), from
    point 0, and each one's squared distance to the nearest earlier one. Returns (order int32 [m],
    dist2 float32 [m]); the initial scale of point order[i] is sqrt(dist2[i])."""
    device = points.device
    _check_dev("points", points, device, torch.float32)
    n = points.shape[0]
    size = ctypes.c_size_t()
    L.check(ctx.lib.nx_fps_workspace_size(n, ctypes.byref(size)))
    ws = torch.empty(int(size.value), device=device, dtype=torch.uint8)
    order = torch.empty(int(m), device=device, dtype=torch.int32)
    d2 = torch.empty(int(m), device=device, dtype=torch.float32)
    stream = ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)
    L.check(ctx.lib.nx_fps(ctx.handle, _ptr(points), n, int(m), _ptr(order), _ptr(d2), _ptr(ws), ws.numel(), stream))
    return order, d2


def densify(ctx: Context, surfels, blended_error, exp_draws, n_split, min_opacity=0.005):
    """nx_densify: split n_split surfels drawn in proportion to blended_error (exponential clocks exp_draws [n]),
    then prune opacities below min_opacity. Returns (the six surfel tensors, parent int32) of the new set
    (synchronises the stream once for its size)."""
    device = surfels[0].device
    n = surfels[0].shape[0]
    for nm, t, shp in (("means", surfels[0], (n, 3)), ("quats", surfels[1], (n, 4)), ("scales", surfels[2], (n, 2)),
                       ("opacities", surfels[3], (n,)), ("gammas", surfels[4], (n, 2)), ("colors", surfels[5], (n, 3)),
                       ("blended_error", blended_error, (n,)), ("exp_draws", exp_draws, (n,))):
        _check_dev(nm, t, device, torch.float32, shp)
    s = L.NxSurfels(*[_ptr(t) for t in surfels], n)
    cap = n + max(int(n_split), 0)
    f32 = dict(device=device, dtype=torch.float32)
    outs = [torch.empty(cap, 3, **f32), torch.empty(cap, 4, **f32), torch.empty(cap, 2, **f32),
            torch.empty(cap, **f32), torch.empty(cap, 2, **f32), torch.empty(cap, 3, **f32)]
    parent = torch.empty(cap, device=device, dtype=torch.int32)
    o = L.NxSurfelsOut(*[_ptr(t) for t in outs], _ptr(parent), cap)
    size = ctypes.c_size_t()
    L.check(ctx.lib.nx_densify_workspace_size(n, ctypes.byref(size)))
    ws = torch.empty(int(size.value), device=device, dtype=torch.uint8)
    n_out = ctypes.c_int64()
    stream = ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)
    L.check(ctx.lib.nx_densify(ctx.handle, ctypes.byref(s), _ptr(blended_error), _ptr(exp_draws), int(n_split),
                               float(min_opacity), ctypes.byref(o), ctypes.byref(n_out), _ptr(ws), ws.numel(), stream))
    k = int(n_out.value)
    return tuple(t[:k] for t in outs), parent[:k]


class RenderFunction(torch.autograd.Function):
    """image, weights, tex = RenderFunction.apply(ctx, cam, level_scales, means, quats, scales,
    opacities, gammas, colors, table, w1, w2, w3).

    Gradients flow to the six surfel tensors, the hash table and the three
    MLP matrices; gradients of storage dtypes other than float32 are
    accumulated in float32 and cast by autograd.
    """

    @staticmethod
    def forward(fctx, nctx, cam, level_scales, means, quats, scales, opac, gammas, colors, table, w1, w2, w3):
        surfels = (means, quats, scales, opac, gammas, colors)
        weights = [w1, w2, w3] if nctx.K > 0 else None
        res = render_forward(nctx, surfels, cam, table, level_scales, weights)
        fctx.nctx = nctx
        fctx.res = res
        fctx.level_scales = level_scales
        fctx.save_for_backward(means, quats, scales, opac, gammas, colors, table, w1, w2, w3)
        fctx.mark_non_differentiable(res.plain, res.ids, res.depths, res.t_final)
        return res.image, res.weights, res.tex, res.plain, res.ids, res.depths, res.t_final

    @staticmethod
    def backward(fctx, g_image, g_weights, g_tex, *unused):
        means, quats, scales, opac, gammas, colors, table, w1, w2, w3 = fctx.saved_tensors
        nctx, res = fctx.nctx, fctx.res
        dev = means.device
        z = lambda t: torch.zeros(t.shape, device=dev, dtype=torch.float32)
        grads = {"means": z(means), "quats": z(quats), "scales": z(scales), "opacities": z(opac),
                 "gammas": z(gammas), "colors": z(colors)}
        if nctx.K > 0:
            grads["table"] = z(table)
            grads["mlp"] = [z(w1), z(w2), z(w3)]
        gi = torch.zeros_like(res.image) if g_image is None else g_image.contiguous().float()
        gw = None if g_weights is None or nctx.K == 0 else g_weights.contiguous().float()
        gt = None if g_tex is None or nctx.K == 0 else g_tex.contiguous().float()
        weights = [w1, w2, w3] if nctx.K > 0 else None
        render_backward(nctx, (means, quats, scales, opac, gammas, colors), res, table, fctx.level_scales, weights,
                        gi, gw, gt, grads)
        gmlp = grads.get("mlp") or [None, None, None]
        return (None, None, None, grads["means"], grads["quats"], grads["scales"], grads["opacities"],
                grads["gammas"], grads["colors"], grads.get("table"), gmlp[0], gmlp[1], gmlp[2])


def render(nctx, cam, level_scales, means, quats, scales, opac, gammas, colors, table, w1, w2, w3):
    """Differentiable render: returns (image [P,3], weights [P,K], tex [P,K,3], plain, ids, depths, t_final)."""
    return RenderFunction.apply(nctx, cam, level_scales, means, quats, scales, opac, gammas, colors, table, w1, w2,
                                w3)
