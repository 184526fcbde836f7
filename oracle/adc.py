"""Adaptive density control (oracle): initialisation, split selection, split and prune.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper, supplementary, Adaptive Density Control (and Optimization, Adaptive
Density Control):
  * Initialisation: farthest point sampling orders the input points so that
    each next point maximises the distance to the points already taken; the
    initial scale of the i-th point is its distance to the nearest earlier
    one, min_{j<i} d(x_{I_i}, x_{I_j}).
  * Densification: per-surfel blended errors, summed over iterations, are
    normalised into probability weights, and a fixed fraction of the
    surfels (5%) is drawn for splitting; the number added is capped so that
    the total stays within the primitive budget.
  * Split: with s1 >= s2 the surfel becomes two with scales (s1 / 2, s2) and
    centres mu -/+ (s1 / 2) v1; every other property (rotation, opacity,
    gamma, colour) is copied. For gamma -> infinity this halves the quad
    along its long axis.
  * Prune: surfels whose opacity is below 0.005 are removed.

Readings (the paper does not settle these):
  * FPS starts at point 0; the distance compared is the squared Euclidean
    distance evaluated in float32 as (dx*dx + dy*dy) + dz*dz with every
    operation rounded (the index it selects is an integer decision, taken
    in the same precision as the kernel); ties go to the smallest index.
    The first point has no predecessor and takes the second point's scale.
  * Weighted sampling without replacement is done with exponential clocks
    (Efraimidis-Spirakis): given draws e_i ~ Exp(1) (passed in), surfel i
    gets the key e_i / w_i (float32 division) and the k smallest keys are
    drawn; this draws in proportion to w without replacement, and the
    normalisation of w does not change the order. Surfels with w <= 0 are
    never drawn; ties go to the smaller index.
  * The long axis is v1 when s1 >= s2, else v2 (the surfel's axes are not
    reordered); the first child keeps the surfel's slot, the second is
    appended after the surviving inputs in input order.
  * Pruning keeps the order of the survivors.
"""
from __future__ import annotations

import numpy as np


def _d2_f32(p, q):
    """Squared distance in float32: (dx*dx + dy*dy) + dz*dz, each operation rounded."""
    d = (np.asarray(p, np.float32) - np.asarray(q, np.float32)).astype(np.float32)
    return (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]).astype(np.float32) + (d[..., 2] * d[..., 2]).astype(np.float32)


def farthest_point_sampling(points, m):
    """Returns (order [m] int64, d2 [m] float32): the FPS order of the first m points and each one's squared
    distance to the nearest earlier point (d2[0] = d2[1])."""
    x = np.asarray(points, np.float32)
    n = x.shape[0]
    m = min(int(m), n)
    order = np.zeros(m, np.int64)
    d2 = np.zeros(m, np.float32)
    if m == 0:
        return order, d2
    best = np.full(n, np.inf, np.float32)
    cur = 0
    for i in range(m):
        order[i] = cur
        d2[i] = best[cur] if i > 0 else np.float32(0.0)
        dist = _d2_f32(x, x[cur])
        best = np.minimum(best, dist).astype(np.float32)
        best[order[: i + 1]] = -1.0  # taken points are never chosen again
        if i + 1 < m:
            cur = int(np.argmax(best))  # first index of the maximum
    if m > 1:
        d2[0] = d2[1]
    return order, d2


def select_splits(errors, exp_draws, k):
    """Indices (sorted ascending) of the k surfels drawn for splitting: the k smallest keys e_i / w_i over the
    surfels with w_i > 0 (ties: smaller index first)."""
    w = np.asarray(errors, np.float32)
    e = np.asarray(exp_draws, np.float32)
    ok = w > 0
    key = np.full(w.shape, np.inf, np.float32)
    key[ok] = (e[ok] / w[ok]).astype(np.float32)
    idx = np.arange(w.shape[0])
    cand = idx[ok]
    order = cand[np.lexsort((cand, key[cand]))]
    return np.sort(order[: min(int(k), order.shape[0])])


def split_and_prune(means, quats, scales, opacities, gammas, colors, chosen, min_opacity=0.005):
    """Split the surfels in `chosen`, then prune. Returns (the six arrays, parent [n_out] int64)."""
    means = np.asarray(means, np.float64)
    quats = np.asarray(quats, np.float64)
    scales = np.asarray(scales, np.float64)
    n = means.shape[0]
    chosen = np.asarray(sorted(chosen), np.int64)
    from .geometry import quat_columns  # the textbook rotation the renderer uses
    import torch
    v1, v2, _ = quat_columns(torch.as_tensor(quats))
    v1, v2 = v1.numpy(), v2.numpy()
    M = [means.copy(), quats.copy(), scales.copy(), np.asarray(opacities, np.float64).copy(),
         np.asarray(gammas, np.float64).copy(), np.asarray(colors, np.float64).copy()]
    parent = list(range(n))
    extra = [[] for _ in range(6)]
    for i in chosen:
        s1, s2 = scales[i]
        if s1 >= s2:
            half, axis, which = s1 / 2.0, v1[i], 0
        else:
            half, axis, which = s2 / 2.0, v2[i], 1
        child_s = scales[i].copy()
        child_s[which] = half
        a = means[i] - half * axis
        b = means[i] + half * axis
        M[0][i] = a
        M[2][i] = child_s
        vals = [b, quats[i], child_s, M[3][i], M[4][i], M[5][i]]
        for k in range(6):
            extra[k].append(vals[k])
        parent.append(int(i))
    out = [np.concatenate([M[k], np.asarray(extra[k]).reshape((-1,) + M[k].shape[1:])]) if extra[k] else M[k]
           for k in range(6)]
    parent = np.asarray(parent, np.int64)
    keep = out[3] >= min_opacity
    return [a[keep] for a in out], parent[keep]
