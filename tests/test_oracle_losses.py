"""Pins of the oracle's auxiliary losses (CPU).

Paper, Optimization, Losses: L_texture, L_alpha, L_opacity, L_grid. Pinned by
closed forms on hand-made inputs, by the scale invariance of the
non-premultiplied texture (its loss is homogeneous of degree 0 in the slot
weights, so sum_j W_j dL/dW_j = 0 per pixel), and by central finite
differences of each loss away from the kinks of |x|.
"""
from __future__ import annotations

import numpy as np

from oracle.losses import aux_losses


def _rand(seed, P=40, K=4, N=30, L=3, T=16):
    rng = np.random.default_rng(seed)
    W = rng.uniform(0.01, 0.3, (P, K))
    X = rng.uniform(0.0, 1.0, (P, K, 3))
    G = rng.uniform(0.0, 1.0, (P, 3))
    o = rng.uniform(0.0, 1.0, N)
    H = rng.uniform(-1.0, 1.0, (L, T, 2))
    s = 16.0 * 1.5 ** np.arange(L) / 16.0
    return W, X, G, o, H, s


def test_closed_forms():
    W = np.array([[0.2, 0.6], [0.0, 0.0]])
    X = np.array([[[0.3, 0.5, 0.9], [0.3, 0.5, 0.9]], [[0.7, 0.7, 0.7], [0.1, 0.1, 0.1]]])
    G = np.array([[0.1, 0.5, 1.0], [0.0, 0.0, 0.0]])
    o = np.array([0.25, 0.75, 0.5, 1.0])
    H = np.full((2, 8, 2), 0.5)
    s = np.array([2.0, 4.0])
    losses, grads = aux_losses(W, X, G, o, H, s)
    # equal textures: the non-premultiplied texture is that texture; the empty pixel adds nothing
    assert abs(losses["texture"] - (0.2 + 0.0 + 0.1) / 6.0) < 1e-15
    assert abs(losses["alpha"] - ((1.0 - 0.8) + 1.0) / 2.0) < 1e-15
    assert abs(losses["opacity"] - 2.5 / 4.0) < 1e-15
    assert abs(losses["grid"] - (2.0 ** -3 + 4.0 ** -3) * 8 * 2 * 0.25) < 1e-15
    assert np.allclose(grads["alpha"]["weights"], -0.5)
    assert np.allclose(grads["opacity"]["opacities"], 0.25)
    assert np.allclose(grads["grid"]["table"][0], 2.0 * 2.0 ** -3 * 0.5)
    assert np.allclose(grads["grid"]["table"][1], 2.0 * 4.0 ** -3 * 0.5)
    # the empty pixel's texture terms have no gradient
    assert np.all(grads["texture"]["weights"][1] == 0.0) and np.all(grads["texture"]["tex"][1] == 0.0)
    # texture gradient of pixel 0: r = X, d|G - r|/dr = -sign(G - r), dr/dTex_j = W_j / S
    sg = -np.sign(G[0] - X[0, 0])
    assert np.allclose(grads["texture"]["tex"][0, 0], sg * (0.2 / 0.8) / 6.0)
    assert np.allclose(grads["texture"]["tex"][0, 1], sg * (0.6 / 0.8) / 6.0)


def test_texture_loss_is_scale_invariant_in_the_weights():
    W, X, G, o, H, s = _rand(0)
    _, grads = aux_losses(W, X, G, o, H, s)
    euler = (W * grads["texture"]["weights"]).sum(axis=1)
    assert np.abs(euler).max() < 1e-15
    # and the loss itself does not move when a pixel's weights are scaled
    l0, _ = aux_losses(W, X, G, o, H, s)
    W2 = W.copy()
    W2[::3] *= 3.7
    l1, _ = aux_losses(W2, X, G, o, H, s)
    assert abs(l0["texture"] - l1["texture"]) < 1e-14


def test_gradients_match_finite_differences():
    W, X, G, o, H, s = _rand(1, P=12, K=2, N=5, L=2, T=4)
    losses, grads = aux_losses(W, X, G, o, H, s)
    h = 1e-7
    cases = [("alpha", "weights", W, 0), ("texture", "weights", W, 0), ("texture", "tex", X, 1),
             ("opacity", "opacities", o, 3), ("grid", "table", H, 4)]
    for loss, name, arr, pos in cases:
        g = grads[loss][name]
        flat = arr.reshape(-1)
        for idx in range(flat.size):
            args = [W, X, G, o, H, s]
            a_p = arr.copy().reshape(-1)
            a_m = arr.copy().reshape(-1)
            a_p[idx] += h
            a_m[idx] -= h
            args[pos] = a_p.reshape(arr.shape)
            lp, _ = aux_losses(*args)
            args[pos] = a_m.reshape(arr.shape)
            lm, _ = aux_losses(*args)
            fd = (lp[loss] - lm[loss]) / (2 * h)
            assert abs(fd - g.reshape(-1)[idx]) <= 1e-6 * max(1.0, abs(fd)), (loss, name, idx, fd, g.reshape(-1)[idx])
