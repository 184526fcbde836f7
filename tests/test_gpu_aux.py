"""Auxiliary losses (nx_aux_losses) against the FP64 oracle (needs an MI355X).

Paper, Optimization, Losses: L_alpha, L_texture, L_opacity, L_grid. Inputs:
the weights and textures of a real forward (the 128x128 / 2000-surfel
workload) and random ones with empty pixels (all weights zero), tables in
FP32, FP16 and BF16. Loss values within 2e-6 relative; every gradient
element within 1e-5 max(|g|, rms(g)) of the oracle's (FP32 arithmetic on
O(1) inputs). Gradients accumulate into the caller's buffers (+=).
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import scenes
from oracle.losses import aux_losses as oracle_aux
from tests.gpu_helpers import device_inputs, log

pytestmark = pytest.mark.gpu

LAMBDAS = (0.3, 0.7, 0.05, 2.0)


@pytest.fixture(scope="module")
def nx():
    import paper_2512_13796_amd as m
    return m


def _check(nx, ctx, W, X, G, o, table, scales, label):
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).float().to(dev)
    Wd, Xd, Gd, od = t(W), t(X), t(G), t(o)
    tab = table.to(dev).contiguous()
    pre = 1e-7  # gradients add to what the buffers hold (small: the float32 sum keeps their digits)
    grads = {"weights": torch.full(Wd.shape, pre, device=dev), "tex": torch.full(Xd.shape, pre, device=dev),
             "opacities": torch.full(od.shape, pre, device=dev),
             "table": torch.full(tab.shape, pre, device=dev, dtype=torch.float32)}
    losses = nx.aux_losses(ctx, Wd, Xd, Gd, od, tab, torch.as_tensor(scales), LAMBDAS, grads)
    torch.cuda.synchronize()
    ol, og = oracle_aux(W, X, G, o, table.float().numpy(), scales)
    got = losses.cpu().numpy().astype(np.float64)
    want = np.array([ol["alpha"], ol["texture"], ol["opacity"], ol["grid"]])
    log(label, "losses", got, "oracle", want)
    assert np.allclose(got, want, rtol=2e-6, atol=1e-9), label
    lam = dict(zip(("alpha", "texture", "opacity", "grid"), LAMBDAS))
    expect = {"weights": lam["alpha"] * og["alpha"]["weights"] + lam["texture"] * og["texture"]["weights"],
              "tex": lam["texture"] * og["texture"]["tex"], "opacities": lam["opacity"] * og["opacity"]["opacities"],
              "table": lam["grid"] * og["grid"]["table"]}
    for k, e in expect.items():
        g = grads[k].cpu().numpy().astype(np.float64) - pre
        scale = max(float(np.sqrt(np.mean(e ** 2))), 1e-30)
        err = np.abs(g - e) / np.maximum(np.abs(e), scale)
        log(label, k, f"max rel err {err.max():.2e}")
        assert err.max() <= 1e-5, f"{label}: {k} max rel err {err.max():.3e}"


@pytest.mark.parametrize("dtype", [torch.float32, torch.float16, torch.bfloat16])
def test_aux_losses_random(nx, dtype):
    rng = np.random.default_rng(3)
    P, K, N = 5000, 4, 3000
    W = rng.uniform(0.0, 0.4, (P, K))
    W[rng.random(P) < 0.1] = 0.0  # empty pixels
    X = rng.uniform(0.0, 1.0, (P, K, 3))
    G = rng.uniform(0.0, 1.0, (P, 3))
    o = rng.uniform(0.0, 1.0, N)
    table = torch.from_numpy(rng.uniform(-1.0, 1.0, (8, 1 << 10, 2))).to(dtype)
    scales = (16.0 * 1.5 ** np.arange(8)).astype(np.float32)
    ctx = nx.Context(K, dtype, torch.float32)
    _check(nx, ctx, W, X, G, o, table, scales, f"random {dtype}")


def test_aux_losses_of_a_forward(nx):
    wl = scenes.make_workload(1)
    surf, table, weights = device_inputs(wl)
    ctx = nx.Context(wl.K, table.dtype, weights[0].dtype)
    res = nx.render_forward(ctx, surf, wl.cameras[0], table, wl.grid.level_scales, weights)
    torch.cuda.synchronize()
    W = res.weights.double().cpu().numpy()
    X = res.tex.double().cpu().numpy()
    G = wl.target[0].reshape(-1, 3).double().numpy() if wl.target[0] is not None else np.zeros((W.shape[0], 3))
    _check(nx, ctx, W, X, G, wl.scene.opacities.double().numpy(), wl.grid.table,
           np.asarray(wl.grid.level_scales, dtype=np.float32), "c1 forward")


@pytest.mark.parametrize("K", [1, 8, 16])
def test_aux_losses_other_slot_counts(nx, K):
    rng = np.random.default_rng(10 + K)
    P, N = 3000, 500
    W = rng.uniform(0.0, 0.4 / K * 4, (P, K))
    W[rng.random(P) < 0.1] = 0.0
    X = rng.uniform(0.0, 1.0, (P, K, 3))
    G = rng.uniform(0.0, 1.0, (P, 3))
    o = rng.uniform(0.0, 1.0, N)
    table = torch.from_numpy(rng.uniform(-1.0, 1.0, (4, 1 << 8, 2))).float()
    scales = (16.0 * 1.5 ** np.arange(4)).astype(np.float32)
    ctx = nx.Context(K, torch.float32, torch.float32)
    _check(nx, ctx, W, X, G, o, table, scales, f"K={K}")
