"""Pins of the oracle's adaptive density control (CPU).

Supplementary, Adaptive Density Control. FPS: a closed-form order on
collinear points, the non-increasing sequence of selection distances, and
the covering property (after m picks every point lies within the next
selection distance of the picked set). Split selection: weights of zero are
never drawn, and over many draws a surfel's chance of being drawn first is
its share of the weights. Split: closed-form children for both long axes and
a rotated surfel, and for gamma -> infinity the two children render the
parent's quad (the split halves a flat-topped quad exactly). Prune:
survivors keep their order and parents.
"""
from __future__ import annotations

import numpy as np
import torch

import oracle
import scenes
from oracle.adc import farthest_point_sampling, select_splits, split_and_prune


def test_fps_collinear_closed_form():
    x = np.zeros((11, 3), np.float32)
    x[:, 0] = np.arange(11)
    order, d2 = farthest_point_sampling(x, 5)
    assert order.tolist() == [0, 10, 5, 2, 7]
    assert d2.tolist() == [100.0, 100.0, 25.0, 4.0, 4.0]


def test_fps_invariants():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(300, 3)).astype(np.float32)
    order, d2 = farthest_point_sampling(x, 300)
    assert sorted(order.tolist()) == list(range(300))
    assert np.all(np.diff(d2[1:]) <= 0.0)
    xd = x.astype(np.float64)
    for m in (1, 5, 40, 150):
        dist = ((xd[:, None, :] - xd[None, order[:m], :]) ** 2).sum(-1).min(axis=1)
        assert abs(dist.max() - d2[m]) <= 1e-5 * max(d2[m], 1e-6)
        assert np.argmax(dist) == order[m]


def test_selection_weights_and_exclusions():
    rng = np.random.default_rng(1)
    w = np.array([0.0, 1.0, 2.0, 3.0, 4.0, 0.0], np.float32)
    counts = np.zeros(6)
    trials = 20000
    for _ in range(trials):
        e = rng.exponential(size=6).astype(np.float32)
        counts[select_splits(w, e, 1)[0]] += 1
    assert counts[0] == 0 and counts[5] == 0
    p = w / w.sum()
    sd = np.sqrt(p * (1 - p) / trials)
    assert np.all(np.abs(counts / trials - p) <= 4 * sd + 1e-12)
    # k beyond the positive weights: every positive one, nothing else
    assert select_splits(w, np.ones(6, np.float32), 10).tolist() == [1, 2, 3, 4]
    # equal keys: the smaller index first
    assert select_splits(np.ones(4, np.float32), np.ones(4, np.float32), 2).tolist() == [0, 1]


def _one(scale, quat=(1.0, 0.0, 0.0, 0.0), mean=(0.0, 0.0, 0.0)):
    return ([list(mean)], [list(quat)], [list(scale)], [0.8], [[1.0, 1.0]], [[0.2, 0.4, 0.6]])


def test_split_closed_forms():
    out, parent = split_and_prune(*_one((0.4, 0.1)), chosen=[0])
    assert np.allclose(out[0], [[-0.2, 0, 0], [0.2, 0, 0]]) and np.allclose(out[2], [[0.2, 0.1]] * 2)
    out, _ = split_and_prune(*_one((0.1, 0.4)), chosen=[0])
    assert np.allclose(out[0], [[0, -0.2, 0], [0, 0.2, 0]]) and np.allclose(out[2], [[0.1, 0.2]] * 2)
    c, s = np.cos(np.pi / 4), np.sin(np.pi / 4)  # +90 degrees about z: v1 = +y
    out, _ = split_and_prune(*_one((0.4, 0.1), quat=(c, 0.0, 0.0, s), mean=(1.0, 2.0, 3.0)), chosen=[0])
    assert np.allclose(out[0], [[1.0, 1.8, 3.0], [1.0, 2.2, 3.0]])
    assert parent.tolist() == [0, 0]
    for k in (1, 3, 4, 5):
        assert np.allclose(out[k][0], out[k][1])


def test_split_halves_a_flat_topped_quad():
    # a facing surfel with gamma = 50 (nearly the quad |u|, |v| <= 1) against its two halves
    quat = (1.0, 0.0, 0.0, 0.0)
    m, q, s, o, g, col = _one((0.3, 0.12), quat=quat, mean=(0.05, -0.02, 0.0))
    g = [[50.0, 50.0]]
    (m2, q2, s2, o2, g2, c2), _ = split_and_prune(m, q, s, o, g, col, chosen=[0])
    cam = scenes.look_at((0.0, 0.0, -2.0), (0.0, 0.0, 0.0), (0.0, -1.0, 0.0), 64, 64)
    grid = scenes.HashGrid(torch.zeros(1, 16, 2), torch.tensor([1.0]))
    mlp = scenes.MLP([torch.zeros(64, 2), torch.zeros(64, 64), torch.zeros(3, 64)])
    f = lambda a: torch.tensor(np.asarray(a), dtype=torch.float32)
    parent = oracle.render(scenes.Scene(f(m), f(q), f(s), f(o), f(g), f(col)), cam, grid, mlp, 0).image
    halves = oracle.render(scenes.Scene(f(m2), f(q2), f(s2), f(o2), f(g2), f(c2)), cam, grid, mlp, 0).image
    diff = np.abs(parent - halves).max(axis=1).reshape(64, 64)
    # pixels away from the seam and the outline agree; the seam is one pixel column
    assert (diff > 1e-3).sum() <= 64 * 2
    assert np.abs(parent.sum() - halves.sum()) <= 0.02 * parent.sum()


def test_prune_keeps_order_and_parents():
    rng = np.random.default_rng(2)
    n = 20
    m = rng.normal(size=(n, 3))
    q = np.tile([1.0, 0, 0, 0], (n, 1))
    s = rng.uniform(0.1, 0.5, (n, 2))
    o = rng.uniform(0.0, 0.02, n)
    out, parent = split_and_prune(m, q, s, o, np.ones((n, 2)), rng.uniform(size=(n, 3)), chosen=[3, 7])
    keep_in = [i for i in range(n) if o[i] >= 0.005]
    extra = [i for i in (3, 7) if o[i] >= 0.005]
    assert parent.tolist() == keep_in + extra
    assert np.all(out[3] >= 0.005)
