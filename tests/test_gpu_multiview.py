"""Several cameras in one call (n_cams > 1) against one call per camera and
against the FP64 oracle.

Workload: the 300k-surfel planes scene with 16 orbit cameras of mixed
resolutions, shrunk to 40k surfels; the first five cameras are rendered
together (640x480 up to 1920x1080 in one call). Per-camera outputs must equal
the single-camera calls bit for bit (same kernels, same inputs); the
gradients of the joint backward must equal the sum of the single-camera
backwards up to float32 summation order; and on a pixel sample per camera
the joint call must match the oracle (forward within 1e-5, gradients summed
over the cameras within the parity bars).
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import scenes
from tests.gpu_helpers import (SAFETY, check_forced_decisions, compare_forward, device_inputs, fmt_grad_report,
                               grad_errors, log, to_np)
from tests.test_gpu_parity import _sample_pixels

pytestmark = pytest.mark.gpu
N_CAMS = 5


@pytest.fixture(scope="module")
def nx():
    import paper_2512_13796_amd as m
    return m


@pytest.fixture(scope="module")
def setup(nx):
    wl = scenes.make_workload(4, seed=0, n_surfels=40_000)
    cams = wl.cameras[:N_CAMS]
    surf, table, weights = device_inputs(wl)
    ctx = nx.Context(wl.K, table.dtype, weights[0].dtype)
    res = nx.render_forward(ctx, surf, cams, table, wl.grid.level_scales, weights, want_cells=True)
    torch.cuda.synchronize()
    return wl, cams, surf, table, weights, ctx, res


def _offsets(cams):
    off = [0]
    for c in cams:
        off.append(off[-1] + c.width * c.height)
    return off


def _zero_grads(surf, table, weights):
    z = lambda t: torch.zeros(t.shape, device=t.device, dtype=torch.float32)
    return {"means": z(surf[0]), "quats": z(surf[1]), "scales": z(surf[2]), "opacities": z(surf[3]),
            "gammas": z(surf[4]), "colors": z(surf[5]), "table": z(table), "mlp": [z(w) for w in weights]}


def test_joint_forward_equals_single_camera_calls(nx, setup):
    wl, cams, surf, table, weights, ctx, res = setup
    off = _offsets(cams)
    log("multi-view resolutions", [(c.width, c.height) for c in cams], "instances", res.n_instances_cam)
    for i, cam in enumerate(cams):
        one = nx.render_forward(ctx, surf, cam, table, wl.grid.level_scales, weights)
        torch.cuda.synchronize()
        sl = slice(off[i], off[i + 1])
        assert one.n_instances == res.n_instances_cam[i]
        for nm in ("image", "plain", "ids", "weights", "depths", "t_final", "tex", "n_iter"):
            a, b = getattr(res, nm)[sl], getattr(one, nm)
            assert torch.equal(a, b), f"camera {i}: {nm} differs from the single-camera call"


def test_joint_backward_equals_sum_of_single_camera_backwards(nx, setup):
    wl, cams, surf, table, weights, ctx, res = setup
    P = res.image.shape[0]
    gen = torch.Generator(device="cuda").manual_seed(3)
    gi = torch.randn(P, 3, device="cuda", generator=gen) * 1e-3
    joint = _zero_grads(surf, table, weights)
    nx.render_backward(ctx, surf, res, table, wl.grid.level_scales, weights, gi, None, None, joint)
    single = _zero_grads(surf, table, weights)
    off = _offsets(cams)
    for i, cam in enumerate(cams):
        one = nx.render_forward(ctx, surf, cam, table, wl.grid.level_scales, weights)
        nx.render_backward(ctx, surf, one, table, wl.grid.level_scales, weights,
                           gi[off[i]:off[i + 1]].contiguous(), None, None, single)
    torch.cuda.synchronize()
    for nm in ("means", "quats", "scales", "opacities", "gammas", "colors", "table"):
        a, b = joint[nm].double(), single[nm].double()
        rel = float((a - b).norm() / max(float(b.norm()), 1e-30))
        assert rel <= 1e-5, f"{nm}: joint vs summed single-camera gradients rel {rel:.2e}"
    for i in range(3):
        a, b = joint["mlp"][i].double(), single["mlp"][i].double()
        rel = float((a - b).norm() / max(float(b.norm()), 1e-30))
        assert rel <= 1e-5, f"mlp{i}: rel {rel:.2e}"


def test_joint_call_against_oracle(nx, setup):
    wl, cams, surf, table, weights, ctx, res = setup
    off = _offsets(cams)
    K = wl.K
    gpu = to_np(res, K)
    grid = scenes.HashGrid(table.cpu(), wl.grid.level_scales)
    mlp = scenes.MLP([w.cpu() for w in weights])
    P = res.image.shape[0]
    rng = np.random.default_rng(11)
    gi = np.zeros((P, 3))
    per_cam = []
    for i, cam in enumerate(cams):
        pix = _sample_pixels(cam, 20 + i, per_block=96, full_tiles=1)
        glob = pix + off[i]
        cells = res.cells[torch.from_numpy(glob).cuda()].cpu().numpy()
        masks = res.relu_masks[torch.from_numpy(glob).cuda()].cpu().numpy().view(np.uint32)
        feats = res.features[torch.from_numpy(glob).cuda()].cpu().numpy()
        nat = oracle.render(wl.scene, cam, grid, mlp, K, pixels=pix, want_decisions=True)
        log(f"cam {i} decisions:", check_forced_decisions(nat, cells, masks, feats, gpu["depths"][glob], cam,
                                                          wl.grid.level_scales, weights, "f32", label=f"cam {i}"))
        orc = oracle.render(wl.scene, cam, grid, mlp, K, pixels=pix, force_cells=cells, force_relu=masks)
        sub = {k: v[off[i]:off[i + 1]] for k, v in gpu.items()}
        stats = compare_forward(sub, orc, pix, K, label=f"cam {i}")
        log(f"multi-view cam {i} ({cam.width}x{cam.height}):", stats)
        dec = orc.margin > SAFETY
        gi[glob[dec]] = rng.standard_normal((int(dec.sum()), 3))
        per_cam.append((cam, pix, cells, masks))
    grads = _zero_grads(surf, table, weights)
    nx.render_backward(ctx, surf, res, table, wl.grid.level_scales, weights,
                       torch.from_numpy(gi).float().cuda(), None, None, grads)
    torch.cuda.synchronize()
    total = None
    for i, (cam, pix, cells, masks) in enumerate(per_cam):
        og = oracle.render_and_grad(wl.scene, cam, grid, mlp, K, pixels=pix, grad_image=gi[pix + off[i]],
                                    force_cells=cells, force_relu=masks).grads
        if total is None:
            total = {k: (v if k != "mlp" else list(v)) for k, v in og.items()}
        else:
            for k, v in og.items():
                if k == "mlp":
                    total[k] = [a + b for a, b in zip(total[k], v)]
                else:
                    total[k] = total[k] + v
    report = {nm: grad_errors(grads[nm].cpu().numpy(), total[nm])
              for nm in ("means", "quats", "scales", "opacities", "gammas", "colors", "table")}
    for i in range(3):
        report[f"mlp{i}"] = grad_errors(grads["mlp"][i].cpu().numpy(), total["mlp"][i])
    log("multi-view grads:", fmt_grad_report(report))
    for k, r in report.items():
        assert r["rel_l2"] <= 1e-3 and r["viol_coarse"] <= 5e-3, f"{k}: {fmt_grad_report({k: r})}"


def test_full_size_all_cameras_against_oracle(nx):
    """The multi-view workload at full size, as bench.py times it (300k surfels, all 16 cameras in one call,
    FP32 grid and MLP): forward within 1e-5 and gradients within the FP32 parity bars on a pixel sample of
    every camera."""
    wl = scenes.make_workload(4)
    cams = wl.cameras
    surf, table, weights = device_inputs(wl)
    ctx = nx.Context(wl.K, table.dtype, weights[0].dtype)
    res = nx.render_forward(ctx, surf, cams, table, wl.grid.level_scales, weights, want_cells=True)
    torch.cuda.synchronize()
    off = _offsets(cams)
    K = wl.K
    gpu = to_np(res, K)
    grid = scenes.HashGrid(table.cpu(), wl.grid.level_scales)
    mlp = scenes.MLP([w.cpu() for w in weights])
    rng = np.random.default_rng(17)
    gi = np.zeros((res.image.shape[0], 3))
    per_cam = []
    n_nd = 0
    for i, cam in enumerate(cams):
        pix = _sample_pixels(cam, 40 + i, per_block=96, full_tiles=0)
        glob = pix + off[i]
        cells = res.cells[torch.from_numpy(glob).cuda()].cpu().numpy()
        masks = res.relu_masks[torch.from_numpy(glob).cuda()].cpu().numpy().view(np.uint32)
        feats = res.features[torch.from_numpy(glob).cuda()].cpu().numpy()
        nat = oracle.render(wl.scene, cam, grid, mlp, K, pixels=pix, want_decisions=True)
        log(f"full-size cam {i} decisions:",
            check_forced_decisions(nat, cells, masks, feats, gpu["depths"][glob], cam, wl.grid.level_scales, weights,
                                   "f32", label=f"full-size cam {i}"))
        orc = oracle.render(wl.scene, cam, grid, mlp, K, pixels=pix, force_cells=cells, force_relu=masks)
        sub = {k: v[off[i]:off[i + 1]] for k, v in gpu.items()}
        # the fraction of pixels within FP32 error of a decision is checked over all cameras below
        compare_forward(sub, orc, pix, K, max_nondecisive=1.0, label=f"full-size cam {i}")
        dec = orc.margin > SAFETY
        n_nd += int((~dec).sum())
        gi[glob[dec]] = rng.standard_normal((int(dec.sum()), 3))
        per_cam.append((cam, pix, cells, masks))
    n_pix = sum(p[1].shape[0] for p in per_cam)
    log(f"full-size multi-view: {n_pix} sampled pixels over {len(cams)} cameras, {n_nd} within FP32 error of a decision")
    assert n_nd <= 1e-2 * n_pix, f"non-decisive pixels {n_nd} of {n_pix}"
    grads = _zero_grads(surf, table, weights)
    nx.render_backward(ctx, surf, res, table, wl.grid.level_scales, weights,
                       torch.from_numpy(gi).float().cuda(), None, None, grads)
    torch.cuda.synchronize()
    total = None
    for i, (cam, pix, cells, masks) in enumerate(per_cam):
        og = oracle.render_and_grad(wl.scene, cam, grid, mlp, K, pixels=pix, grad_image=gi[pix + off[i]],
                                    force_cells=cells, force_relu=masks).grads
        if total is None:
            total = {k: (v if k != "mlp" else list(v)) for k, v in og.items()}
        else:
            for k, v in og.items():
                total[k] = [a + b for a, b in zip(total[k], v)] if k == "mlp" else total[k] + v
    report = {nm: grad_errors(grads[nm].cpu().numpy(), total[nm])
              for nm in ("means", "quats", "scales", "opacities", "gammas", "colors", "table")}
    for i in range(3):
        report[f"mlp{i}"] = grad_errors(grads["mlp"][i].cpu().numpy(), total["mlp"][i])
    log("full-size multi-view grads:", fmt_grad_report(report))
    for k, r in report.items():
        assert r["rel_l2"] <= 1e-3 and r["viol_coarse"] <= 5e-3, f"{k}: {fmt_grad_report({k: r})}"


def test_joint_call_with_tiny_and_ragged_cameras(nx, setup):
    """Cameras of very different sizes in one call (a 7x5 and a 1x1 view between larger ones, ragged edges):
    the joint binning launch numbers their blocks camera after camera, so every camera boundary falls inside
    a workgroup's share. Forward outputs equal the single-camera calls bit for bit, gradients their sum."""
    import dataclasses
    wl, cams0, surf, table, weights, ctx, _ = setup
    sizes = [(7, 5), (333, 211), (1, 1), (640, 480)]
    cams = []
    for (w, h), c in zip(sizes, cams0):
        f = c.fx * w / c.width
        cams.append(dataclasses.replace(c, width=w, height=h, fx=f, fy=f, cx=w / 2.0, cy=h / 2.0))
    res = nx.render_forward(ctx, surf, cams, table, wl.grid.level_scales, weights)
    P = res.image.shape[0]
    gi = torch.randn(P, 3, device="cuda", generator=torch.Generator(device="cuda").manual_seed(11))
    joint = _zero_grads(surf, table, weights)
    nx.render_backward(ctx, surf, res, table, wl.grid.level_scales, weights, gi, None, None, joint)
    single = _zero_grads(surf, table, weights)
    off = _offsets(cams)
    for i, cam in enumerate(cams):
        one = nx.render_forward(ctx, surf, cam, table, wl.grid.level_scales, weights)
        torch.cuda.synchronize()
        for nm in ("image", "plain", "weights", "depths", "t_final", "tex"):
            a = getattr(res, nm)[off[i]:off[i + 1]]
            assert torch.equal(a, getattr(one, nm)), f"camera {i} ({cam.width}x{cam.height}): {nm}"
        nx.render_backward(ctx, surf, one, table, wl.grid.level_scales, weights,
                           gi[off[i]:off[i + 1]].contiguous(), None, None, single)
    torch.cuda.synchronize()
    for nm in ("means", "quats", "scales", "opacities", "gammas", "colors", "table"):
        a, b = joint[nm].double(), single[nm].double()
        rel = float((a - b).norm() / max(float(b.norm()), 1e-30))
        log(f"tiny/ragged cameras: {nm} joint vs single rel {rel:.2e}")
        # float32 atomic order only (random upstream gradients: the sums cancel, differences reach ~1e-5)
        assert rel <= 1e-4, f"{nm}: joint vs summed single-camera gradients rel {rel:.2e}"
