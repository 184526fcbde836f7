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
    ctx = nx.Context(K, table.dtype, weights[0].dtype, sh_degree=getattr(wl, "sh_degree", None))
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


# Per-element bound of the BF16 form's gradients, relative to max(|g|, rms(g)): every matrix-core operand is
# rounded to BF16 (relative error 2^-9) in each of the MLP's three forward and three backward products, and the
# surfel and table gradients inherit those errors through dL/dW, dL/dD and the feature gradients; 16 roundings
# of 2^-9 give 2^-5.
BF16_ELEM = 2.0 ** -5


def grad_errors(g_gpu, g_orc):
    """Error statistics of one gradient tensor against the oracle's.

    rel_l2      ||g_gpu - g||_2 / ||g||_2
    viol        fraction of elements over 1e-3 max(|g|, 1e-2 rms(g)) (the
                per-element rule)
    viol_coarse fraction over 1e-3 max(|g|, 1e-1 rms(g))
    viol_bf16   fraction over BF16_ELEM max(|g|, rms(g)) (the BF16 form's rule)
    max_abs, mean_abs, rms  absolute errors and the tensor's own rms."""
    g_gpu = np.asarray(g_gpu, dtype=np.float64).reshape(-1)
    g_orc = np.asarray(g_orc, dtype=np.float64).reshape(-1)
    diff = np.abs(g_gpu - g_orc)
    norm = np.linalg.norm(g_orc)
    rel_l2 = float(np.linalg.norm(g_gpu - g_orc) / norm) if norm > 0 else float(np.linalg.norm(g_gpu))
    rms = math.sqrt(float(np.mean(g_orc ** 2))) if g_orc.size else 0.0
    n = max(diff.size, 1)
    return {"rel_l2": rel_l2,
            "viol": float(np.sum(diff > 1e-3 * np.maximum(np.abs(g_orc), 1e-2 * rms))) / n,
            "viol_coarse": float(np.sum(diff > 1e-3 * np.maximum(np.abs(g_orc), 1e-1 * rms))) / n,
            "viol_bf16": float(np.sum(diff > BF16_ELEM * np.maximum(np.abs(g_orc), rms))) / n,
            "max_abs": float(diff.max()) if diff.size else 0.0, "mean_abs": float(diff.mean()) if diff.size else 0.0,
            "rms": rms}


def fmt_grad_report(rep):
    return {k: f"rel {v['rel_l2']:.2e} viol {v['viol']:.1e}/{v['viol_coarse']:.1e}/{v.get('viol_bf16', 0):.1e} "
               f"max {v['max_abs']:.2e} mean {v['mean_abs']:.2e} rms {v['rms']:.2e}" for k, v in rep.items()}


# Relative error scales of the MLP pre-activations per layer, as inputs to the
# decision check: FP32 matrix cores accumulate at most 128 products (a few
# units of 2^-24 of sum |W x|); BF16 matrix cores see inputs rounded to BF16
# (2^-9 each) and accumulate in FP32.
MLP_REL_ERR = {"f32": 4e-6, "bf16": 2.0 ** -8}


def check_forced_decisions(orc, gpu_cells, gpu_masks, gpu_feats, gpu_depths, cam, level_scales, weights, form,
                           label="", feat_tol=1e-5, table_absmax=None):
    """Check the decisions the kernel reported against the FP64 oracle's own.

    orc must come from oracle.render(..., want_decisions=True) on the same
    pixels (decisive pixels only are checked; there the ids agree).
      * Hash cell per slot, level and axis: equal to floor(s_l x) of the
        oracle's FP64 point x = o + D d, unless that coordinate lies within
        its FP32 error bound of a cell face (then off by one towards it).
        Bound (two times): |s_l D d_a| |D_gpu - D| / D (the depth the kernel
        was given) + 4e-7 s_l D |d| (ray direction) + 2e-7 (|s_l D d_a| + 1)
        (FP32 rounding of the camera-relative coordinate) + 1e-6.
      * Features z: within feat_tol max(1, max|z|) of the oracle's FP64 ones,
        plus (given table_absmax, the largest |entry|) the change the FP32
        error of the lattice point can make: trilinear interpolation moves a
        feature by at most 2 table_absmax per cell per axis, so
        2 table_absmax sum_axis (the cell bound above) per level.
      * ReLU bit per hidden unit: equal to the sign of the FP64 pre-activation
        of the natural network, unless |pre| is within two times its error
        bound: layer 1 e1 = |W1| |z_gpu - z| + r |W1| |z|, layer 2
        e2 = |W2| (e1 + r |h1|) + r |W2| |h1| (r = MLP_REL_ERR[form]).
    Returns the counts; raises AssertionError on a decision outside its band."""
    from oracle.mlp import hidden_preactivations

    dec = (orc.margin > SAFETY)
    K = orc.ids.shape[1]
    has = (orc.ids >= 0) & dec[:, None]
    stats = {"slots": int(has.sum())}
    if stats["slots"] == 0:
        return stats
    L = orc.lattice.shape[2]
    m = np.asarray(cam.world_to_cam, dtype=np.float64)
    o_world = -m[:, :3].T @ m[:, 3]
    s = np.asarray(level_scales, dtype=np.float64)
    lat = orc.lattice[has]                                   # [n, L, 3]
    D = orc.depths[has]                                      # [n]
    Dg = np.asarray(gpu_depths, dtype=np.float64)[has]
    cells = np.asarray(gpu_cells, dtype=np.int64)[has]       # [n, L, 3]
    nat = np.floor(lat).astype(np.int64)
    sDd = lat - s[None, :, None] * o_world[None, None, :]
    sD = s[None, :] * D[:, None]                             # [n, L]
    dnorm = np.linalg.norm(sDd, axis=2) / sD
    bound = 2.0 * (np.abs(sDd) * (np.abs(Dg - D) / D)[:, None, None] + 4e-7 * (sD * dnorm)[:, :, None]
                   + 2e-7 * (np.abs(sDd) + 1.0) + 1e-6)
    diff = cells != nat
    up_ok = (cells == nat + 1) & (nat + 1 - lat <= bound)
    dn_ok = (cells == nat - 1) & (lat - nat <= bound)
    bad = diff & ~(up_ok | dn_ok)
    stats.update(cell_coords=int(diff.size), cell_diff=int(diff.sum()), cell_bad=int(bad.sum()),
                 cell_near_face=int((np.minimum(lat - nat, nat + 1 - lat) <= bound).sum()))
    if bad.any():
        i = np.argwhere(bad)[:3]
        raise AssertionError(f"{label}: hash cell differs from floor(s_l x) away from a face at "
                             f"{[(tuple(x), float(lat[tuple(x)]), int(cells[tuple(x)]), float(bound[tuple(x)])) for x in i]}")
    z = orc.features[has]
    zg = np.asarray(gpu_feats, dtype=np.float64)[has]
    ferr = np.abs(zg - z)
    stats["feat_max_err"] = float(ferr.max())
    tol = np.full(z.shape, feat_tol * max(1.0, float(np.abs(z).max())))
    if table_absmax is not None:
        F = z.shape[1] // L
        pos = 2.0 * float(table_absmax) * bound.sum(axis=2)           # [n, L]
        tol = tol + np.repeat(pos, F, axis=1)
    worst = float((ferr / tol).max())
    stats["feat_err_over_bound"] = worst
    assert worst <= 1.0, f"{label}: feature error {stats['feat_max_err']:.3e} beyond its bound ({worst:.2f}x)"
    r = MLP_REL_ERR[form]
    W = [np.asarray(w.detach().cpu().double().numpy() if hasattr(w, "detach") else w, dtype=np.float64)
         for w in weights]
    pre1, pre2 = hidden_preactivations(z, W)
    h1 = np.maximum(pre1, 0.0)
    e1 = ferr @ np.abs(W[0]).T + r * (np.abs(z) @ np.abs(W[0]).T)
    e2 = (e1 + r * h1) @ np.abs(W[1]).T + r * (h1 @ np.abs(W[1]).T)
    H = W[0].shape[0]
    words = np.asarray(gpu_masks).astype(np.uint32)[has].reshape(-1, 2, H // 32)
    bits = ((words[:, :, :, None] >> np.arange(32, dtype=np.uint32)) & 1).reshape(-1, 2, H).astype(bool)
    out = {}
    for li, (pre, e) in enumerate(((pre1, e1), (pre2, e2))):
        nat_bit = pre > 0
        d = bits[:, li] != nat_bit
        band = np.abs(pre) <= 2.0 * e
        out[li] = (int(d.sum()), int((d & ~band).sum()), int(band.sum()))
        if (d & ~band).any():
            i = np.argwhere(d & ~band)[:3]
            raise AssertionError(f"{label}: ReLU layer {li + 1} bit differs from the FP64 sign outside its error "
                                 f"band at {[(tuple(x), float(pre[tuple(x)]), float(e[tuple(x)])) for x in i]}")
    stats.update(relu_units=int(pre1.size + pre2.size), relu_diff=out[0][0] + out[1][0],
                 relu_band=out[0][2] + out[1][2])
    return stats
