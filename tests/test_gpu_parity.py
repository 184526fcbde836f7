"""HIP path against the FP64 oracle (needs an MI355X).

Every call goes through the C ABI (nx_render_forward / nx_render_backward)
via the ctypes binding. Sizes: the 128x128 workload and smaller variants are
compared in full; the 1024x768 and 1920x1080 workloads are compared on a
stratified pixel sample (the oracle evaluates each sampled pixel against
every surfel), with gradients driven by an upstream gradient that is zero
outside the sample so both sides compute the same quantity.

Bars: tile keys, tile lists and per-pixel top-K ids bit-exact (ids on
decisive pixels); FP32 outputs within 1e-5; gradients within 1e-3 relative
(L2 per tensor); the BF16/FP16 form at PSNR >= 45 dB against the oracle.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import scenes
from oracle.binning import bin_surfels
from tests.gpu_helpers import (BF16_ELEM, SAFETY, TOL_IMAGE, check_forced_decisions, compare_forward, device_inputs,
                               fmt_grad_report, grad_errors, log, psnr, run_forward, to_np)

pytestmark = pytest.mark.gpu

# BF16 form, per element: |g_gpu - g| <= BF16_ELEM max(|g|, rms(g)) (tests.gpu_helpers: 2^-5 from sixteen BF16
# roundings of 2^-9); at most this fraction of a tensor's elements may exceed it, for the elements whose
# gradient is a sum of contributions that cancel (their error follows the contributions, not the sum).
BF16_VIOL = 1e-3


@pytest.fixture(scope="module")
def nx():
    import paper_2512_13796_amd as nx
    return nx


def _ws_view(res, off, count, dtype):
    b = res.workspace[off:off + count * 4]
    return b.view(dtype).cpu().numpy()


def _check_binning(nx, wl, label):
    ctx, surf, table, weights, res = run_forward(nx, wl)
    cam = wl.cameras[0]
    n = wl.scene.n
    info = bin_surfels(wl.scene, cam)
    lay = ctx.workspace_layout(n, cam, res.n_instances)
    keys = _ws_view(res, lay["depth_keys"], n, torch.int32).view(np.uint32)
    counts = _ws_view(res, lay["tile_counts"], n, torch.int32)
    rects = _ws_view(res, lay["rects"], 4 * n, torch.int32).reshape(n, 4)
    I = res.n_instances
    log(f"{label}: n={n} instances={I} oracle={info['tiles'].shape[0]}")
    alive = info["alive"]
    np.testing.assert_array_equal(keys[alive], info["key"][alive].view(np.uint32))
    np.testing.assert_array_equal(counts, info["count"])
    has = info["count"] > 0
    np.testing.assert_array_equal(rects[has], info["rect"][has])
    assert I == info["tiles"].shape[0]
    tiles = _ws_view(res, lay["sorted_tiles"], I, torch.int32)
    ids = _ws_view(res, lay["sorted_ids"], I, torch.int32)
    np.testing.assert_array_equal(tiles, info["tiles"])
    np.testing.assert_array_equal(ids, info["ids"])
    nt = info["ntx"] * info["nty"]
    rng = _ws_view(res, lay["tile_ranges"], 2 * nt, torch.int32).reshape(nt, 2)
    nonempty = info["ranges"][:, 1] > info["ranges"][:, 0]
    np.testing.assert_array_equal(rng[nonempty], info["ranges"][nonempty])
    assert np.all(rng[~nonempty, 0] == rng[~nonempty, 1])


def test_binning_bit_exact_small(nx):
    _check_binning(nx, scenes.make_workload(1), "c1")


def test_binning_bit_exact_near_plane_crossing(nx):
    wl = scenes.make_workload(1, seed=5, n_surfels=3000, width=53, height=37)
    wl.cameras = [scenes.look_at((0.0, 0.0, -0.3), (0.0, 0.0, 1.0), (0.0, -1.0, 0.0), 53, 37)]
    _check_binning(nx, wl, "near-plane")


def test_binning_bit_exact_outdoor_full_size(nx):
    _check_binning(nx, scenes.make_workload(3), "c3")


def _forward_case(nx, wl, K=None, label="", max_nd=1e-3, feat_dtype=None, mlp_dtype=None, pixels=None,
                  want_cells=True, tol=TOL_IMAGE):
    """Forward parity at decisive pixels; with want_cells (K > 0) the kernel's hash cells, features and ReLU
    decisions are checked against the oracle's natural FP64 ones and then imposed on the oracle, so that the
    forward and gradients are compared on the same branch."""
    K = wl.K if K is None else K
    want_cells = want_cells and K > 0
    ctx, surf, table, weights, res = run_forward(nx, wl, feat_dtype, mlp_dtype, K=K, want_cells=want_cells)
    gpu = to_np(res, K)
    cam = wl.cameras[0]
    grid = scenes.HashGrid(table.cpu(), wl.grid.level_scales)
    mlp = scenes.MLP([w.cpu() for w in weights])
    if pixels is None:
        pixels = np.arange(cam.width * cam.height)
    cells = masks = None
    if want_cells:
        sel = torch.from_numpy(pixels).to(res.cells.device)
        cells = res.cells[sel].cpu().numpy()
        masks = res.relu_masks[sel].cpu().numpy().view(np.uint32)
        feats = res.features[sel].cpu().numpy()
        nat = oracle.render(wl.scene, cam, grid, mlp, K, pixels=pixels, want_decisions=True, sh_degree=wl.sh_degree)
        form = "bf16" if weights[0].dtype == torch.bfloat16 else "f32"
        dstats = check_forced_decisions(nat, cells, masks, feats, gpu["depths"][pixels], cam, wl.grid.level_scales,
                                        weights, form, label=label, table_absmax=float(table.float().abs().max()))
        log(label, "decisions:", dstats)
    orc = oracle.render(wl.scene, cam, grid, mlp, K, pixels=pixels, force_cells=cells, force_relu=masks,
                        sh_degree=wl.sh_degree)
    stats = compare_forward(gpu, orc, pixels, K, tol=tol, tol_tex=tol, max_nondecisive=max_nd, label=label)
    log(label, stats)
    return ctx, surf, table, weights, res, gpu, orc, (cells, masks)


def test_forward_small_full_frame(nx):
    _forward_case(nx, scenes.make_workload(1), label="c1 fwd")


@pytest.mark.parametrize("K", [0, 1, 2, 8, 16])
def test_forward_other_k(nx, K):
    _forward_case(nx, scenes.make_workload(1, seed=1, width=64, height=64), K=K, label=f"c1 K={K}")


def test_forward_generalised_gamma(nx):
    wl = scenes.make_workload(1, seed=2, width=64, height=64)
    g = np.random.default_rng(2).uniform(1.0, 8.0, (wl.scene.n, 2)).astype(np.float32)
    wl.scene.gammas = torch.from_numpy(g)
    _forward_case(nx, wl, label="gamma")


def test_forward_ragged_image(nx):
    _forward_case(nx, scenes.make_workload(1, seed=3, width=37, height=23), label="37x23")


def test_forward_near_plane_crossing(nx):
    wl = scenes.make_workload(1, seed=5, n_surfels=3000, width=53, height=37)
    wl.cameras = [scenes.look_at((0.0, 0.0, -0.3), (0.0, 0.0, 1.0), (0.0, -1.0, 0.0), 53, 37)]
    _forward_case(nx, wl, label="near-plane", max_nd=5e-3)


def test_forward_empty_and_culled(nx):
    # no surfels at all
    wl = scenes.make_workload(1, seed=4, width=32, height=32, n_surfels=1)
    for sc in (scenes.Scene(*[t[:0] for t in wl.scene.tensors()]),):
        wl.scene = sc
        ctx, surf, table, weights, res = run_forward(nx, wl)
        assert res.n_instances == 0
        assert torch.all(res.image == 0) and torch.all(res.t_final == 1) and torch.all(res.ids == -1)
    # every surfel behind the camera or with a non-positive scale or NaN
    wl = scenes.make_workload(1, seed=4, width=32, height=32, n_surfels=50)
    m = wl.scene.means.clone()
    m[:, 2] = -5.0
    wl.scene.means = m
    s = wl.scene.scales.clone()
    s[:10, 0] = 0.0
    wl.scene.scales = s
    o = wl.scene.opacities.clone()
    o[10:20] = float("nan")
    wl.scene.opacities = o
    ctx, surf, table, weights, res = run_forward(nx, wl)
    assert res.n_instances == 0
    assert torch.all(res.image == 0) and torch.all(res.ids == -1)


def test_forward_deterministic(nx):
    wl = scenes.make_workload(1, seed=6)
    a = run_forward(nx, wl)[4]
    b = run_forward(nx, wl)[4]
    for k in ("image", "plain", "ids", "weights", "depths", "t_final", "tex", "n_iter"):
        assert torch.equal(getattr(a, k), getattr(b, k)), k


def _grad_case(nx, wl, K=None, label="", feat_dtype=None, mlp_dtype=None, pixels=None, rel_tol=1e-3,
               viol_tol=5e-3, with_aux=True, tol_fwd=TOL_IMAGE, max_nd=1e-3, bf16_bound=None):
    K = wl.K if K is None else K
    ctx, surf, table, weights, res, gpu, orc, forced = _forward_case(nx, wl, K=K, label=label + " fwd",
                                                                    feat_dtype=feat_dtype, mlp_dtype=mlp_dtype,
                                                                    pixels=pixels, want_cells=True, tol=tol_fwd,
                                                                    max_nd=max_nd)
    cam = wl.cameras[0]
    P = cam.width * cam.height
    if pixels is None:
        pixels = np.arange(P)
    rng = np.random.default_rng(123)
    # the oracle evaluates the hash cells and ReLU branches the kernel took
    decisive = orc.margin > SAFETY
    log(label, f"gradient pixels excluded: {1.0 - decisive.mean():.2e}, ReLU decisions within FP32 error: "
               f"{(orc.mlp_margin <= SAFETY).mean():.2e} of pixels")
    mask = np.zeros(P)
    mask[pixels[decisive]] = 1.0
    gi = rng.standard_normal((P, 3)) * mask[:, None]
    gw = rng.standard_normal((P, max(K, 1))) * mask[:, None] if (with_aux and K > 0) else None
    gt = rng.standard_normal((P, max(K, 1), 3)) * mask[:, None, None] if (with_aux and K > 0) else None
    dev = surf[0].device
    z = lambda t: torch.zeros(t.shape, device=dev, dtype=torch.float32)
    grads = {"means": z(surf[0]), "quats": z(surf[1]), "scales": z(surf[2]), "opacities": z(surf[3]),
             "gammas": z(surf[4]), "colors": z(surf[5])}
    if K > 0:
        grads["table"] = z(table)
        grads["mlp"] = [z(w) for w in weights]
    f = lambda a: None if a is None else torch.from_numpy(a).float().to(dev).contiguous()
    # densification signal: blended errors of a per-pixel error map on the same pixels
    perr = np.abs(rng.standard_normal(P)) * mask
    grads["blended_error"] = torch.zeros(wl.scene.n, device=dev, dtype=torch.float32)
    nx.render_backward(ctx, surf, res, table, wl.grid.level_scales, weights if K > 0 else None,
                       f(gi), f(gw), f(gt), grads, pixel_error=f(perr))
    torch.cuda.synchronize()
    grid = scenes.HashGrid(table.cpu(), wl.grid.level_scales)
    mlp = scenes.MLP([w.cpu() for w in weights])
    og = oracle.render_and_grad(wl.scene, cam, grid, mlp, K, pixels=pixels, grad_image=gi[pixels],
                                grad_weights=None if gw is None else gw[pixels],
                                grad_tex=None if gt is None else gt[pixels], force_cells=forced[0],
                                force_relu=forced[1], pixel_error=perr[pixels], sh_degree=wl.sh_degree)
    blended = og.blended_error
    og = og.grads
    report = {}
    names = ["means", "quats", "scales", "opacities", "gammas", "colors"] + (["table"] if K > 0 else [])
    for nm in names:
        report[nm] = grad_errors(grads[nm].cpu().numpy(), og[nm])
    if K > 0:
        for i in range(3):
            report[f"mlp{i}"] = grad_errors(grads["mlp"][i].cpu().numpy(), og["mlp"][i])
    be = grad_errors(grads["blended_error"].cpu().numpy(), blended)
    log(label, "blended error:", fmt_grad_report({"blended": be}))
    assert be["rel_l2"] <= 1e-5 and be["viol"] == 0.0, f"{label}: blended error {fmt_grad_report({'b': be})}"
    log(label, "grad:", fmt_grad_report(report))
    for k, r in report.items():
        assert r["rel_l2"] <= rel_tol, f"{label}: {k} rel L2 {r['rel_l2']:.3e} > {rel_tol}"
        if bf16_bound is None:
            # FP32 form: every element within 1e-3 max(|g|, 1e-2 rms) but for a fraction viol_tol. An MLP
            # weight-gradient element sums one term per sample (thousands), and with random upstream gradients
            # the terms cancel (the sum is about n^-1/2 of their magnitudes), so FP32 accumulation leaves every
            # element an absolute error of 1e-5 to 1e-4 rms whatever its size: for them the floor is 1e-1 rms.
            viol = r["viol_coarse"] if k.startswith("mlp") else r["viol"]
            assert viol <= viol_tol, f"{label}: {k} per-element violations {viol:.3e}"
        else:
            # BF16 operands: elements within BF16_ELEM max(|g|, rms(g)), but for a fraction bf16_bound
            assert r["viol_bf16"] <= bf16_bound, \
                f"{label}: {k}: {r['viol_bf16']:.2e} of the elements beyond {BF16_ELEM} max(|g|, rms)"
    return report


def test_backward_small_full_frame(nx):
    _grad_case(nx, scenes.make_workload(1), label="c1")


def test_backward_generalised_gamma(nx):
    wl = scenes.make_workload(1, seed=2, width=64, height=64)
    g = np.random.default_rng(2).uniform(1.0, 8.0, (wl.scene.n, 2)).astype(np.float32)
    wl.scene.gammas = torch.from_numpy(g)
    _grad_case(nx, wl, label="gamma")


@pytest.mark.parametrize("K", [0, 1, 8])
def test_backward_other_k(nx, K):
    _grad_case(nx, scenes.make_workload(1, seed=7, width=48, height=40), K=K, label=f"K={K}")


def test_backward_hidden128_fp32(nx):
    """MLP 32-128-128-3 (the 1M-surfel 1440p workload's width) on a small view, FP32 form, K=8."""
    wl = scenes.make_workload(5, seed=9, n_surfels=40_000, width=160, height=90, feat_dtype=torch.float32,
                              mlp_dtype=torch.float32)
    pix = _sample_pixels(wl.cameras[0], 3, per_block=16, full_tiles=2)
    _grad_case(nx, wl, label="h128 fp32", pixels=pix)


def test_backward_hidden128_bf16(nx):
    """Same, BF16 grid and BF16 MLP: activations are rounded to BF16 (unit roundoff 2^-8) between the
    three layers, so gradients carry a relative error of a few 2^-8; bound 5e-2 on the relative L2."""
    wl = scenes.make_workload(5, seed=10, n_surfels=40_000, width=160, height=90)
    pix = _sample_pixels(wl.cameras[0], 4, per_block=16, full_tiles=2)
    _grad_case(nx, wl, label="h128 bf16", pixels=pix, rel_tol=5e-2, bf16_bound=BF16_VIOL, tol_fwd=1e-3)


def test_autograd_function_matches_direct_call(nx):
    wl = scenes.make_workload(1, seed=8, width=48, height=48)
    surf, table, weights = device_inputs(wl)
    ctx = nx.Context(wl.K, table.dtype, weights[0].dtype)
    leaves = [t.clone().requires_grad_(True) for t in surf]
    tbl = table.clone().requires_grad_(True)
    ws = [w.clone().requires_grad_(True) for w in weights]
    img, W, tex, *_ = nx.render(ctx, wl.cameras[0], wl.grid.level_scales, *leaves, tbl, *ws)
    target = torch.rand_like(img)
    loss = ((img - target) ** 2).mean()
    loss.backward()
    res = nx.render_forward(ctx, surf, wl.cameras[0], table, wl.grid.level_scales, weights)
    gi = (2.0 * (res.image - target) / img.numel()).contiguous()
    z = lambda t: torch.zeros(t.shape, device=t.device, dtype=torch.float32)
    grads = {"means": z(surf[0]), "quats": z(surf[1]), "scales": z(surf[2]), "opacities": z(surf[3]),
             "gammas": z(surf[4]), "colors": z(surf[5]), "table": z(table), "mlp": [z(w) for w in weights]}
    nx.render_backward(ctx, surf, res, table, wl.grid.level_scales, weights, gi, None, None, grads)
    torch.cuda.synchronize()
    for leaf, nm in zip(leaves, ["means", "quats", "scales", "opacities", "gammas", "colors"]):
        np.testing.assert_allclose(leaf.grad.cpu().numpy(), grads[nm].cpu().numpy(), rtol=1e-4, atol=1e-9)
    np.testing.assert_allclose(tbl.grad.cpu().numpy(), grads["table"].cpu().numpy(), rtol=1e-4, atol=1e-9)


def _sample_pixels(cam, seed, per_block=32, full_tiles=1):
    """One random pixel per per_block x per_block block plus full 16x16 tiles."""
    rng = np.random.default_rng(seed)
    pix = []
    for by in range(0, cam.height, per_block):
        for bx in range(0, cam.width, per_block):
            x = bx + rng.integers(0, min(per_block, cam.width - bx))
            y = by + rng.integers(0, min(per_block, cam.height - by))
            pix.append(y * cam.width + x)
    ntx = (cam.width + 15) // 16
    nty = (cam.height + 15) // 16
    for t in rng.choice(ntx * nty, full_tiles, replace=False):
        tx, ty = t % ntx, t // ntx
        for y in range(ty * 16, min(ty * 16 + 16, cam.height)):
            for x in range(tx * 16, min(tx * 16 + 16, cam.width)):
                pix.append(y * cam.width + x)
    return np.unique(np.array(pix, dtype=np.int64))


def test_forward_indoor_sampled(nx):
    wl = scenes.make_workload(2)
    pix = _sample_pixels(wl.cameras[0], 0, per_block=32, full_tiles=2)
    log(f"c2 sampled pixels: {pix.shape[0]}")
    _forward_case(nx, wl, label="c2 fwd", pixels=pix)


def test_outdoor_fp32_form_sampled(nx):
    wl = scenes.make_workload(3, feat_dtype=torch.float32, mlp_dtype=torch.float32)
    pix = _sample_pixels(wl.cameras[0], 1, per_block=64, full_tiles=2)
    log(f"c3 fp32 sampled pixels: {pix.shape[0]}")
    _grad_case(nx, wl, label="c3 fp32", pixels=pix)


def test_outdoor_bf16_form_gradients_sampled(nx):
    """FP16 grid + BF16 MLP at 1080p: gradient errors per tensor against the FP64 oracle on a pixel sample.
    The MLP runs on BF16 matrix cores (activations rounded to 2^-8 between layers), so the bar is the BF16
    one (relative L2 <= 5e-2); surfel gradients go through no BF16 rounding and stay near FP32 accuracy."""
    wl = scenes.make_workload(3)
    pix = _sample_pixels(wl.cameras[0], 7, per_block=64, full_tiles=2)
    # a pixel sample of ~1500: one pixel within the decision margins is 7e-4 of it
    rep = _grad_case(nx, wl, label="c3 bf16", pixels=pix, rel_tol=5e-2, bf16_bound=BF16_VIOL, tol_fwd=1e-3,
                     max_nd=3e-3)
    for nm in ("means", "quats", "scales", "opacities", "gammas", "colors"):
        assert rep[nm]["rel_l2"] <= 1e-3, f"{nm}: {rep[nm]['rel_l2']:.2e}"


def test_large_hidden128_bf16_gradients_sampled(nx):
    """The large workload at full size, as bench.py times it: 1M surfels, 2560x1440, K = 8, BF16 grid and
    hidden-128 BF16 MLP. Forward and gradients against the FP64 oracle on a pixel sample, with the BF16 bars
    of the 1080p test; surfel gradients go through no BF16 rounding and stay near FP32 accuracy."""
    wl = scenes.make_workload(5)
    pix = _sample_pixels(wl.cameras[0], 13, per_block=96, full_tiles=1)
    log(f"c5 sampled pixels: {pix.shape[0]}")
    rep = _grad_case(nx, wl, label="c5 bf16", pixels=pix, rel_tol=5e-2, bf16_bound=BF16_VIOL, tol_fwd=1e-3,
                     max_nd=1e-2)
    for nm in ("means", "quats", "scales", "opacities", "gammas", "colors"):
        assert rep[nm]["rel_l2"] <= 1e-3, f"{nm}: {rep[nm]['rel_l2']:.2e}"


def test_outdoor_bf16_form_psnr(nx):
    """FP16 grid + BF16 MLP: image PSNR against the FP64 oracle >= 45 dB."""
    wl = scenes.make_workload(3)
    pix = _sample_pixels(wl.cameras[0], 2, per_block=96)
    ctx, surf, table, weights, res = run_forward(nx, wl)
    gpu = to_np(res, wl.K)
    grid = scenes.HashGrid(table.cpu(), wl.grid.level_scales)
    mlp = scenes.MLP([w.cpu() for w in weights])
    orc = oracle.render(wl.scene, wl.cameras[0], grid, mlp, wl.K, pixels=pix)
    d = orc.margin > SAFETY
    assert np.array_equal(gpu["ids"][pix][d], orc.ids[d])
    p = psnr(gpu["image"][pix], orc.image)
    err = np.abs(gpu["image"][pix] - orc.image)
    terr = np.abs(gpu["tex"][pix] - orc.tex)[orc.ids >= 0]
    log(f"c3 bf16: PSNR {p:.1f} dB, image max {err.max():.2e} mean {err.mean():.2e}, tex max {terr.max():.2e} "
        f"mean {terr.mean():.2e}")
    assert p >= 45.0


def test_indoor_fp32_gradients_sampled(nx):
    """The indoor workload (100k surfels on planes, 1024x768, K = 4, FP32 grid and MLP) forward and backward on a
    pixel sample, with the FP32 bars."""
    wl = scenes.make_workload(2)
    pix = _sample_pixels(wl.cameras[0], 8, per_block=32, full_tiles=2)
    log(f"c2 fp32 sampled pixels: {pix.shape[0]}")
    _grad_case(nx, wl, label="c2 fp32", pixels=pix)


def test_outdoor_bf16_form_unit_features(nx):
    """BF16 form (FP16 grid, BF16 MLP) at 1080p with table entries U(-1, 1): features of order one, so the BF16
    rounding of the MLP's inputs and activations is not suppressed by tiny features. Image PSNR against the FP64
    oracle >= 45 dB; max and mean absolute errors of the image, the textures and every gradient are reported."""
    wl = scenes.make_workload(3, grid_amp=1.0)
    pix = _sample_pixels(wl.cameras[0], 9, per_block=64, full_tiles=2)
    rep = _grad_case(nx, wl, label="c3 bf16 unit", pixels=pix, rel_tol=5e-2, bf16_bound=BF16_VIOL, tol_fwd=2e-2,
                     max_nd=3e-3)
    ctx, surf, table, weights, res = run_forward(nx, wl)
    gpu = to_np(res, wl.K)
    grid = scenes.HashGrid(table.cpu(), wl.grid.level_scales)
    mlp = scenes.MLP([w.cpu() for w in weights])
    orc = oracle.render(wl.scene, wl.cameras[0], grid, mlp, wl.K, pixels=pix)
    d = orc.margin > SAFETY
    p = psnr(gpu["image"][pix][d], orc.image[d])
    err = np.abs(gpu["image"][pix][d] - orc.image[d])
    terr = np.abs(gpu["tex"][pix][d] - orc.tex[d])[orc.ids[d] >= 0]
    log(f"c3 bf16 unit features: PSNR {p:.1f} dB, image max {err.max():.2e} mean {err.mean():.2e}, "
        f"tex max {terr.max():.2e} mean {terr.mean():.2e}")
    assert p >= 45.0
    return rep


def test_stop_rule_and_clamp_scenes(nx):
    """The hand-built stop-rule stack (five alpha = 0.95 surfels on one ray) and the opacity-1 clamp case, through
    the HIP path against the oracle: three composited, T_final = 0.05^3; alpha clamped at 0.99."""
    from tests.oracle_cases import identity_camera, random_grid, random_mlp, scene_from
    # 32x32: the stack (around pixel (8, 8), reaching 9.3 px from it) and the clamp surfel (around pixel
    # (26, 26), 6.2 px) do not overlap
    cam = identity_camera(32, 32, 20.0)
    dx = (8 + 0.5 - cam.cx) / cam.fx
    zs = [2.0, 2.5, 3.0, 3.5, 4.0, 5.0]
    means = [[z * dx, z * dx, z] for z in zs]
    opac = [0.95] * 5 + [1.0]
    means[5] = [5.0 * (26 + 0.5 - cam.cx) / cam.fx, 5.0 * (26 + 0.5 - cam.cy) / cam.fy, 5.0]
    rng = np.random.default_rng(40)
    # scales chosen so that no pixel centre falls exactly on a support edge |u| = 3 (a tie of the support test)
    sc = scene_from(means, [[1, 0, 0, 0]] * 6, [[0.31, 0.31]] * 5 + [[0.52, 0.52]], opac, [[1, 1]] * 6,
                    rng.uniform(0, 1, (6, 3)), dtype=torch.float32)
    grid = random_grid(rng, levels=8, log2_size=10, scale=0.01)
    grid = scenes.HashGrid(grid.table.float(), grid.level_scales)
    mlp = random_mlp(rng, [16, 64, 64, 3])
    mlp = scenes.MLP([w.float() for w in mlp.weights])
    wl = scenes.Workload("stack", sc, [cam], grid, mlp, 4, [None])
    ctx, surf, table, weights, res, gpu, orc, _ = _forward_case(nx, wl, label="stack")
    p = 8 * 32 + 8
    assert orc.n_comp[p] == 3 and list(gpu["ids"][p]) == [0, 1, 2, -1]
    np.testing.assert_allclose(gpu["t_final"][p], (1.0 - np.float32(0.95)) ** 3, rtol=1e-5)
    q = 26 * 32 + 26
    assert list(gpu["ids"][q]) == [5, -1, -1, -1]
    np.testing.assert_allclose(gpu["t_final"][q], 0.01, rtol=1e-5)


def test_hash_scatter_fallback_paths(nx):
    """The hash-grid gradient's fallbacks, forced with nx_debug_limits: slabs of 4 records (every further record
    of a bucket goes to the table with a float atomic) and one LDS compare-and-swap attempt (a lost race goes to a
    global atomic). The table gradient equals the default path's (itself checked against the oracle by the other
    tests) up to float32 summation order."""
    wl = scenes.make_workload(1, seed=12)
    surf, table, weights = device_inputs(wl)
    ctx = nx.Context(wl.K, table.dtype, weights[0].dtype)
    res = nx.render_forward(ctx, surf, wl.cameras[0], table, wl.grid.level_scales, weights)
    P = res.image.shape[0]
    gi = torch.randn(P, 3, device="cuda", generator=torch.Generator(device="cuda").manual_seed(3))
    out = []
    for limits in ((0, 0), (4, 1)):
        c = nx.Context(wl.K, table.dtype, weights[0].dtype)
        c.debug_limits(*limits)
        g = {"table": torch.zeros(table.shape, device="cuda", dtype=torch.float32)}
        nx.render_backward(c, surf, res, table, wl.grid.level_scales, weights, gi, None, None, g)
        torch.cuda.synchronize()
        out.append(g["table"].double())
    rel = float((out[1] - out[0]).norm() / out[0].norm())
    log(f"fallback paths: table gradient relative difference {rel:.2e}")
    assert rel <= 1e-5
