"""Adaptive density control on the GPU (nx_fps, nx_densify) against the oracle (needs an MI355X).

Supplementary, Adaptive Density Control.
  * FPS: the order and the squared distances are integer / float32
    decisions taken in the same float32 arithmetic on both sides, so they
    must match the oracle bit for bit (clustered points, duplicates, m = 1,
    m = n). At a size the Python oracle cannot finish (200k points, 50k
    taken) the properties that hold at any size are checked: the order is a
    set of distinct indices, the distances never increase, sampled entries
    equal the float32 distance to the nearest earlier point, and at sampled
    steps no point lies farther from the points taken so far.
  * Densify: the surfels drawn, their children and the survivors of the
    prune equal the oracle's bit for bit (parents exact; FP64 child centres
    rounded to float32 on both sides).
"""
from __future__ import annotations

import time

import numpy as np
import pytest
import torch

from oracle.adc import _d2_f32, farthest_point_sampling, select_splits, split_and_prune
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nx():
    import paper_2512_13796_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(nx):
    return nx.Context(0)


def _clustered(rng, n):
    centres = rng.normal(scale=3.0, size=(16, 3))
    return (centres[rng.integers(0, 16, n)] + rng.normal(scale=0.3, size=(n, 3))).astype(np.float32)


def _gpu_fps(nx, ctx, pts, m):
    order, d2 = nx.fps(ctx, torch.from_numpy(pts).cuda(), m)
    torch.cuda.synchronize()
    return order.cpu().numpy().astype(np.int64), d2.cpu().numpy()


@pytest.mark.parametrize("n,m", [(20000, 1500), (300, 300), (50, 1)])
def test_fps_equals_oracle(nx, ctx, n, m):
    rng = np.random.default_rng(n)
    pts = _clustered(rng, n)
    pts[n // 2] = pts[3]  # a duplicate point
    o_gpu, d_gpu = _gpu_fps(nx, ctx, pts, m)
    o_ref, d_ref = farthest_point_sampling(pts, m)
    log(f"fps n={n} m={m}: first {o_gpu[:6].tolist()}, last d2 {d_gpu[-1]:.4g}")
    assert np.array_equal(o_gpu, o_ref)
    assert np.array_equal(d_gpu.view(np.uint32), d_ref.view(np.uint32))


def test_fps_properties_at_size(nx, ctx):
    rng = np.random.default_rng(9)
    n, m = 200_000, 50_000
    pts = _clustered(rng, n)
    t0 = time.perf_counter()
    order, d2 = _gpu_fps(nx, ctx, pts, m)
    dt = time.perf_counter() - t0
    log(f"fps {n} points -> {m}: {dt * 1e3:.0f} ms ({dt / m * 1e6:.1f} us per point taken)")
    assert len(np.unique(order)) == m and order.min() >= 0 and order.max() < n
    assert np.all(np.diff(d2[1:]) <= 0.0)
    for i in rng.choice(np.arange(1, m), 20, replace=False):
        dd = _d2_f32(pts[order[:i]], pts[order[i]]).min()
        assert dd == d2[i], (i, dd, d2[i])
    for i in (1, 2, 17, 200):
        best = np.full(n, np.inf, np.float32)
        for j in order[:i]:
            best = np.minimum(best, _d2_f32(pts, pts[j]))
        best[order[:i]] = -1.0
        assert best.max() == d2[i] and int(np.argmax(best)) == order[i]


def _scene(rng, n):
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return [rng.normal(size=(n, 3)), q, rng.lognormal(np.log(0.05), 0.5, (n, 2)), rng.uniform(0.0, 0.05, n),
            rng.uniform(1.0, 4.0, (n, 2)), rng.uniform(0.0, 1.0, (n, 3))]


@pytest.mark.parametrize("n,frac", [(5000, 0.05), (777, 0.0), (2000, 0.5)])
def test_densify_equals_oracle(nx, ctx, n, frac):
    rng = np.random.default_rng(n)
    sc = [a.astype(np.float32) for a in _scene(rng, n)]
    err = rng.exponential(size=n).astype(np.float32)
    err[rng.random(n) < 0.2] = 0.0
    draws = rng.exponential(size=n).astype(np.float32)
    k = int(round(frac * n))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    out, parent = nx.densify(ctx, tuple(dev(a) for a in sc), dev(err), dev(draws), k, 0.005)
    chosen = select_splits(err, draws, k)
    ref, ref_parent = split_and_prune(*sc, chosen=chosen, min_opacity=0.005)
    log(f"densify n={n}: {len(chosen)} split, {len(ref_parent)} survive")
    assert np.array_equal(parent.cpu().numpy(), ref_parent)
    for a, b in zip(out, ref):
        assert np.array_equal(a.cpu().numpy(), b.astype(np.float32))


def test_fps_beyond_register_capacity_equals_oracle(nx, ctx):
    """More points than the registers of a full grid hold (256 CUs x 1024 threads x 8 points): FPS keeps the
    nearest distances in global memory instead; the order and distances must still equal the oracle's."""
    rng = np.random.default_rng(21)
    n, m = 2_200_000, 60
    pts = _clustered(rng, n)
    o_gpu, d_gpu = _gpu_fps(nx, ctx, pts, m)
    o_ref, d_ref = farthest_point_sampling(pts, m)
    log(f"fps n={n} m={m} (distances in global memory): last d2 {d_gpu[-1]:.4g}")
    assert np.array_equal(o_gpu, o_ref)
    assert np.array_equal(d_gpu.view(np.uint32), d_ref.view(np.uint32))
