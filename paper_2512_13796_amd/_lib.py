"""ctypes view of the C ABI declared in include/nexels.h.

Loading fails with ImportError when libnexels.so has not been built; there
is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libnexels.so")

NX_OK = 0
NX_ERR_INVALID = -1
NX_ERR_WORKSPACE = -2
NX_ERR_HIP = -3
NX_ERR_UNSUPPORTED = -4

NX_F32, NX_F16, NX_BF16 = 0, 1, 2

c_void_p = ctypes.c_void_p


class NxSurfels(ctypes.Structure):
    _fields_ = [("means", c_void_p), ("quats", c_void_p), ("scales", c_void_p), ("opacities", c_void_p),
                ("gammas", c_void_p), ("colors", c_void_p), ("n", ctypes.c_int64)]


class NxCamera(ctypes.Structure):
    _fields_ = [("world_to_cam", ctypes.c_double * 12), ("fx", ctypes.c_double), ("fy", ctypes.c_double),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double), ("near_z", ctypes.c_double),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class NxHashGrid(ctypes.Structure):
    _fields_ = [("table", c_void_p), ("dtype", ctypes.c_int), ("levels", ctypes.c_int32),
                ("log2_size", ctypes.c_int32), ("feat", ctypes.c_int32), ("level_scales", c_void_p)]


class NxMLP(ctypes.Structure):
    _fields_ = [("w", c_void_p * 3), ("dtype", ctypes.c_int), ("dims", ctypes.c_int32 * 4)]


class NxFwdOut(ctypes.Structure):
    _fields_ = [("image", c_void_p), ("plain", c_void_p), ("ids", c_void_p), ("weights", c_void_p),
                ("depths", c_void_p), ("t_final", c_void_p), ("tex", c_void_p), ("n_iter", c_void_p),
                ("cells", c_void_p), ("relu_masks", c_void_p), ("features", c_void_p),
                ("n_instances", ctypes.POINTER(ctypes.c_int64))]


class NxGrads(ctypes.Structure):
    _fields_ = [("means", c_void_p), ("quats", c_void_p), ("scales", c_void_p), ("opacities", c_void_p),
                ("gammas", c_void_p), ("colors", c_void_p), ("table", c_void_p), ("mlp", c_void_p * 3),
                ("pixel_error", c_void_p), ("blended_error", c_void_p)]


class NxAuxLambdas(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_float), ("texture", ctypes.c_float), ("opacity", ctypes.c_float),
                ("grid", ctypes.c_float)]


class NxSurfelsOut(ctypes.Structure):
    _fields_ = [("means", c_void_p), ("quats", c_void_p), ("scales", c_void_p), ("opacities", c_void_p),
                ("gammas", c_void_p), ("colors", c_void_p), ("parent", c_void_p), ("capacity", ctypes.c_int64)]


class NxWsLayout(ctypes.Structure):
    _fields_ = [(nm, ctypes.c_size_t) for nm in ("depth_keys", "tile_counts", "rects", "records", "sorted_tiles",
                                                  "sorted_ids", "tile_ranges", "total")]


# Every exported symbol with its argument and return types.
SIGNATURES = {
    "nx_version": ([], ctypes.c_int),
    "nx_last_error": ([], ctypes.c_char_p),
    "nx_create": ([ctypes.POINTER(c_void_p), ctypes.c_int32, ctypes.c_int32, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "nx_destroy": ([c_void_p], ctypes.c_int),
    "nx_set_sh_degree": ([c_void_p, ctypes.c_int32], ctypes.c_int),
    "nx_debug_limits": ([c_void_p, ctypes.c_int64, ctypes.c_int32], ctypes.c_int),
    "nx_workspace_size": ([c_void_p, ctypes.c_int64, ctypes.POINTER(NxCamera), ctypes.c_int32, ctypes.c_int64,
                           ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "nx_workspace_size_exact": ([c_void_p, ctypes.POINTER(NxSurfels), ctypes.POINTER(NxCamera), ctypes.c_int32,
                                 c_void_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t),
                                 ctypes.POINTER(ctypes.c_int64), c_void_p], ctypes.c_int),
    "nx_workspace_layout": ([c_void_p, ctypes.c_int64, ctypes.POINTER(NxCamera), ctypes.c_int32, ctypes.c_int64,
                             ctypes.POINTER(NxWsLayout)], ctypes.c_int),
    "nx_render_forward": ([c_void_p, ctypes.POINTER(NxSurfels), ctypes.POINTER(NxCamera), ctypes.c_int32,
                           ctypes.POINTER(NxHashGrid), ctypes.POINTER(NxMLP), ctypes.POINTER(NxFwdOut), c_void_p,
                           ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t), c_void_p], ctypes.c_int),
    "nx_render_backward": ([c_void_p, ctypes.POINTER(NxSurfels), ctypes.POINTER(NxCamera), ctypes.c_int32,
                            ctypes.POINTER(NxHashGrid), ctypes.POINTER(NxMLP), ctypes.POINTER(NxFwdOut), c_void_p,
                            ctypes.c_size_t, c_void_p, c_void_p, c_void_p, ctypes.POINTER(NxGrads), c_void_p],
                           ctypes.c_int),
    "nx_render_forward_async": ([c_void_p, ctypes.POINTER(NxSurfels), ctypes.POINTER(NxCamera), ctypes.c_int32,
                                 ctypes.POINTER(NxHashGrid), ctypes.POINTER(NxMLP), ctypes.POINTER(NxFwdOut),
                                 ctypes.c_int64, c_void_p, ctypes.c_size_t, c_void_p], ctypes.c_int),
    "nx_render_forward_noalloc": ([c_void_p, ctypes.POINTER(NxSurfels), ctypes.POINTER(NxCamera), ctypes.c_int32,
                                   ctypes.POINTER(NxHashGrid), ctypes.POINTER(NxMLP), ctypes.POINTER(NxFwdOut),
                                   ctypes.c_int64, c_void_p], ctypes.c_int),
    "nx_aux_losses": ([c_void_p, ctypes.c_int64, c_void_p, c_void_p, c_void_p, ctypes.c_int64, c_void_p,
                       ctypes.POINTER(NxHashGrid), ctypes.POINTER(NxAuxLambdas), c_void_p, c_void_p, c_void_p,
                       c_void_p, c_void_p, c_void_p], ctypes.c_int),
    "nx_fps_workspace_size": ([ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "nx_fps": ([c_void_p, c_void_p, ctypes.c_int64, ctypes.c_int64, c_void_p, c_void_p, c_void_p, ctypes.c_size_t,
                c_void_p], ctypes.c_int),
    "nx_densify_workspace_size": ([ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "nx_densify": ([c_void_p, ctypes.POINTER(NxSurfels), c_void_p, c_void_p, ctypes.c_int64, ctypes.c_float,
                    ctypes.POINTER(NxSurfelsOut), ctypes.POINTER(ctypes.c_int64), c_void_p, ctypes.c_size_t,
                    c_void_p], ctypes.c_int),
    "nx_autotune_raster": ([c_void_p, ctypes.POINTER(NxSurfels), ctypes.POINTER(NxCamera), ctypes.c_int32,
                            ctypes.POINTER(NxFwdOut), c_void_p, ctypes.c_size_t, ctypes.c_int32,
                            ctypes.POINTER(ctypes.c_int32), c_void_p], ctypes.c_int),
    "nx_instance_counts": ([c_void_p, ctypes.c_int64, ctypes.POINTER(NxCamera), ctypes.c_int32,
                            ctypes.POINTER(ctypes.c_int64), c_void_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_int64),
                            c_void_p], ctypes.c_int),
    "nx_timing_enable": ([c_void_p, ctypes.c_int], ctypes.c_int),
    "nx_timing_reset": ([c_void_p], ctypes.c_int),
    "nx_timing_get": ([c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_double),
                       ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
}

_lib = None


def load():
    """Load libnexels.so once; raise ImportError if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2512_13796_amd/build.py`")
    # torch ships its own HIP runtime. Loaded first, it is the runtime the library binds to (same soname);
    # loaded after the library, a second HIP and HSA runtime would enter the process, and whichever opens the
    # device second finds none.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


class NexelsError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"nexels error {code}: {message}")
        self.code = code


def check(code):
    if code != NX_OK:
        msg = load().nx_last_error().decode(errors="replace")
        raise NexelsError(code, msg)
    return code
