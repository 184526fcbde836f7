"""Shared plumbing for the GPU parity tests: move a workload to the device,
run the HIP path through the C ABI, and compare with the oracle."""
from __future__ import annotations

import math
import sys

import numpy as np
import torch

SAFETY = 2.0          # a decision is trusted if its margin exceeds twice its worst-case FP32 error bound
TOL_IMAGE = 1e-5      # max abs error on image, N, W, T_final, Tex (FP32 form)
TOL_DEPTH_REL = 1e-5  # max relative error on D


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def device_inputs(wl, feat_dtype=None, mlp_dtype=None, device="cuda:0"):
    sc = wl.scene
    surf = tuple(t.to(device).float().contiguous() for t in sc.tensors())
    table = wl.grid.table.to(device)
    if feat_dtype is not None:
        table = table.float().to(feat_dtype)
    weights = [w.to(device) for w in wl.mlp.weights]
    if mlp_dtype is not None:
        weights = [w.float().to(mlp_dtype) for w in weights]
    return surf, table.contiguous(), [w.contiguous() for w in weights]


def host_grid_mlp(table, weights):
    """The exact stored values the device used, for the oracle."""
    import scenes
    grid_t = table.detach().cpu()
    return grid_t, [w.detach().cpu() for w in weights]


def run_forward(nx, wl, feat_dtype=None, mlp_dtype=None, K=None, cam_index=0, want_cells=False):
    surf, table, weights = device_inputs(wl, feat_dtype, mlp_dtype)
    K = wl.K if K is None else K
    ctx = nx.Context(K, table.dtype, weights[0].dtype)
    cam = wl.cameras[cam_index]
    res = nx.render_forward(ctx, surf, cam, table, wl.grid.level_scales, weights, want_cells=want_cells)
    torch.cuda.synchronize()
    return ctx, surf, table, weights, res


def to_np(res, K):
    P = res.image.shape[0]
    out = {
        "image": res.image.double().cpu().numpy(),
        "plain": res.plain.double().cpu().numpy(),
        "t_final": res.t_final.double().cpu().numpy(),
    }
    if K > 0:
        out["ids"] = res.ids.cpu().numpy().astype(np.int64)
        out["weights"] = res.weights.double().cpu().numpy()
        out["depths"] = res.depths.double().cpu().numpy()
        out["tex"] = res.tex.double().cpu().numpy()
    else:
        out["ids"] = np.zeros((P, 0), dtype=np.int64)
        out["weights"] = np.zeros((P, 0))
        out["depths"] = np.zeros((P, 0))
        out["tex"] = np.zeros((P, 0, 3))
    return out


def compare_forward(gpu, orc, pixels, K, tol=TOL_IMAGE, tol_tex=TOL_IMAGE, safety=SAFETY, max_nondecisive=1e-3,
                    label=""):
    """Element-wise comparison at decisive pixels; returns a stats dict."""
    decisive = orc.margin > safety
    nd = 1.0 - decisive.mean()
    stats = {"pixels": int(pixels.shape[0]), "nondecisive_frac": float(nd)}
    g = {k: v[pixels] for k, v in gpu.items()}
    d = decisive
    assert nd <= max_nondecisive, f"{label}: non-decisive fraction {nd:.2e} > {max_nondecisive}"
    ids_ok = np.array_equal(g["ids"][d], orc.ids[d])
    if not ids_ok:
        bad = np.nonzero(np.any(g["ids"][d] != orc.ids[d], axis=1))[0][:5]
        pix = pixels[d][bad]
        raise AssertionError(f"{label}: id mismatch at decisive pixels {pix.tolist()}: gpu {g['ids'][d][bad].tolist()}"
                             f" oracle {orc.ids[d][bad].tolist()} margins {orc.margin[d][bad].tolist()}")
    for key in ("image", "plain", "t_final", "weights", "tex"):
        err = np.abs(g[key][d] - getattr(orc, key)[d])
        stats[f"{key}_max"] = float(err.max()) if err.size else 0.0
        stats[f"{key}_mean"] = float(err.mean()) if err.size else 0.0
        lim = tol_tex if key == "tex" else tol
        assert stats[f"{key}_max"] <= lim, f"{label}: {key} max err {stats[f'{key}_max']:.3e} > {lim}"
    if K > 0:
        dd = g["depths"][d]
        do = orc.depths[d]
        has = orc.ids[d] >= 0
        rel = np.abs(dd[has] - do[has]) / np.abs(do[has])
        stats["depth_rel_max"] = float(rel.max()) if rel.size else 0.0
        assert stats["depth_rel_max"] <= TOL_DEPTH_REL, f"{label}: depth rel err {stats['depth_rel_max']:.3e}"
    return stats


def psnr(a, b):
    mse = float(np.mean((a - b) ** 2))
    return float("inf") if mse == 0 else -10.0 * math.log10(mse)


def grad_errors(g_gpu, g_orc):
    """Per-tensor relative L2 error, and the fraction of elements over the
    per-element bound 1e-3 max(|g|, 0.1 rms(g)).

    The floor at a tenth of the tensor's rms reflects FP32 accumulation over
    thousands of samples: every element carries an absolute error of order
    1e-5 rms(g) whatever its own size, so smaller elements are compared in
    absolute terms."""
    g_gpu = np.asarray(g_gpu, dtype=np.float64).reshape(-1)
    g_orc = np.asarray(g_orc, dtype=np.float64).reshape(-1)
    diff = np.abs(g_gpu - g_orc)
    norm = np.linalg.norm(g_orc)
    rel_l2 = float(np.linalg.norm(g_gpu - g_orc) / norm) if norm > 0 else float(np.linalg.norm(g_gpu))
    rms = math.sqrt(float(np.mean(g_orc ** 2))) if g_orc.size else 0.0
    bound = 1e-3 * np.maximum(np.abs(g_orc), 0.1 * rms)
    viol = float(np.mean(diff > bound)) if diff.size else 0.0
    return rel_l2, viol, float(diff.max()) if diff.size else 0.0
