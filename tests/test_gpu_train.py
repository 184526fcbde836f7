"""Training check: the texture path learns what per-surfel colours cannot.

Targets are rendered by the FP64 oracle from a teacher (hash grid + MLP with
K = 4) on textured planes. Two students with the same geometry start from
fresh colours, grid and MLP and are trained with Adam for 500 steps on six
views through the library's autograd function (forward and backward are the
HIP kernels): one with K = 4 (colours, grid and MLP trained), one with K = 0
(colours only). On the held-out view the K = 4 student must beat the K = 0
student (paper: the texture-limit table, K = 0 against K >= 1). The
gradients of the K = 4 student are checked against the oracle before and
after training.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import scenes
from tests.gpu_helpers import log, psnr
from tests.test_gpu_parity import _grad_case, _sample_pixels

pytestmark = pytest.mark.gpu

STEPS = 500


@pytest.fixture(scope="module")
def nx():
    import paper_2512_13796_amd as m
    return m


@pytest.fixture(scope="module")
def setup():
    tw = scenes.make_train_workload()
    targets = [oracle.render(tw.scene, cam, tw.teacher_grid, tw.teacher_mlp, tw.K).image for cam in tw.cameras]
    return tw, targets


def _student_workload(tw, colors, table, weights, K):
    scene = scenes.Scene(*tw.scene.tensors()[:5], colors.detach().cpu().contiguous())
    grid = scenes.HashGrid(table.detach().cpu().contiguous(), tw.init_grid.level_scales)
    mlp = scenes.MLP([w.detach().cpu().contiguous() for w in weights])
    return scenes.Workload("train", scene, [tw.cameras[0]], grid, mlp, K, [None])


def _train(nx, tw, targets, K):
    dev = torch.device("cuda:0")
    geom = [t.to(dev).contiguous() for t in tw.scene.tensors()[:5]]
    colors = tw.init_colors.to(dev).clone().requires_grad_(True)
    table = tw.init_grid.table.to(dev).clone().requires_grad_(K > 0)
    weights = [w.to(dev).clone().requires_grad_(K > 0) for w in tw.init_mlp.weights]
    ctx = nx.Context(K)
    groups = [{"params": [colors], "lr": 1e-2}]
    if K > 0:
        groups += [{"params": [table], "lr": 1e-2}, {"params": weights, "lr": 2e-3}]
    opt = torch.optim.Adam(groups)
    tgt = [torch.from_numpy(t).float().to(dev) for t in targets]
    n_train = len(tw.cameras) - 1
    ls = tw.init_grid.level_scales
    first = None
    for step in range(STEPS):
        v = step % n_train
        img = nx.render(ctx, tw.cameras[v], ls, *geom, colors, table, *weights)[0]
        loss = ((img - tgt[v]) ** 2).mean()
        opt.zero_grad()
        loss.backward()
        opt.step()
        if first is None:
            first = float(loss.detach())
    with torch.no_grad():
        img = nx.render(ctx, tw.cameras[-1], ls, *geom, colors, table, *weights)[0]
        torch.cuda.synchronize()
        held = psnr(img.double().cpu().numpy(), targets[-1])
    log(f"K={K}: first loss {first:.3e}, last {float(loss.detach()):.3e}, held-out PSNR {held:.2f} dB")
    return held, colors, table, weights


def test_texture_beats_colours_on_held_out_view(nx, setup):
    tw, targets = setup
    # gradients at the student's starting point
    wl0 = _student_workload(tw, tw.init_colors, tw.init_grid.table, tw.init_mlp.weights, tw.K)
    _grad_case(nx, wl0, label="train step 0", pixels=_sample_pixels(wl0.cameras[0], 5, per_block=8))
    p4, colors, table, weights = _train(nx, tw, targets, tw.K)
    p0, *_ = _train(nx, tw, targets, 0)
    # gradients at the trained point
    wl1 = _student_workload(tw, colors, table, weights, tw.K)
    _grad_case(nx, wl1, label=f"train step {STEPS}", pixels=_sample_pixels(wl1.cameras[0], 6, per_block=8))
    # measured: 40.2 dB against 28.8 dB; the bar leaves room for atomic-order differences in training
    assert p4 > p0 + 5.0, f"K=4 held-out PSNR {p4:.2f} dB does not beat K=0 {p0:.2f} dB by 5 dB"
