"""Auxiliary losses of the optimisation and their gradients (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper, Optimization, Losses (H x W pixels p, K texture slots j, channels c):
  L_texture  the non-premultiplied texture should match the ground truth:
             1/(3P) sum_p sum_c | GT_pc - (sum_j W_pj Tex_pjc) / (sum_j W_pj) |
  L_alpha    the non-textured blending weight should vanish:
             1/P sum_p (1 - sum_j W_pj)
  L_opacity  sparsity: 1/N sum_i o_i (o the activated opacity)
  L_grid     grid regularisation, read as sum_l s_l^-3 sum_i sum_f H_lif^2.

Readings (the paper does not settle these):
  * L_grid is printed as a sum of s_i^-3 H_lif, linear in H and indexed by the
    entry i. A linear term has a constant gradient and no minimum, while the
    text says the term keeps grid values near zero mean (to justify the
    down-weighting, after Zip-NeRF); it is read as the level scale s_l and
    squared entries: a weight decay normalised by the level's cell volume.
  * A pixel with sum_j W_pj = 0 has no texture estimate and adds nothing to
    L_texture (nor any gradient).
  * |x| has derivative sign(x), taken as 0 at x = 0.
  * P is the number of pixels passed (several views concatenated form one
    mean).

Gradients are reverse-mode autograd through these FP64 expressions.
"""
from __future__ import annotations

import numpy as np
import torch


def _t(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64))


def aux_losses(weights, tex, target, opacities, table, level_scales):
    """Returns (losses, grads): losses = {alpha, texture, opacity, grid} (floats, unweighted); grads = the
    gradient of each loss w.r.t. its inputs: {alpha: {weights}, texture: {weights, tex}, opacity: {opacities},
    grid: {table}} as float64 arrays. weights [P,K], tex [P,K,3], target [P,3], opacities [N],
    table [L,T,F] (any float dtype; converted exactly), level_scales [L]."""
    W = _t(weights).requires_grad_(True)
    X = _t(tex).requires_grad_(True)
    G = _t(target)
    o = _t(opacities).requires_grad_(True)
    H = torch.as_tensor(table).to(torch.float64).detach().requires_grad_(True)
    s = _t(level_scales)
    P = W.shape[0]

    l_alpha = (1.0 - W.sum(dim=1)).sum() / P

    S = W.sum(dim=1)                              # [P]
    has = S > 0
    Sd = torch.where(has, S, torch.ones_like(S))
    r = (W[:, :, None] * X).sum(dim=1) / Sd[:, None]    # [P,3]
    l_texture = (torch.abs(G - r).sum(dim=1) * has).sum() / (3 * P)

    l_opacity = o.sum() / max(o.shape[0], 1)

    l_grid = (s ** -3.0 * (H * H).sum(dim=(1, 2))).sum()

    (ga_w,) = torch.autograd.grad(l_alpha, [W])
    gt_w, gt_x = torch.autograd.grad(l_texture, [W, X], allow_unused=True)
    (go,) = torch.autograd.grad(l_opacity, [o])
    (gg,) = torch.autograd.grad(l_grid, [H])
    z = lambda a, ref: (torch.zeros_like(ref) if a is None else a).numpy()
    losses = {"alpha": l_alpha.item(), "texture": l_texture.item(), "opacity": l_opacity.item(),
              "grid": l_grid.item()}
    grads = {"alpha": {"weights": ga_w.numpy()},
             "texture": {"weights": z(gt_w, W), "tex": z(gt_x, X)},
             "opacity": {"opacities": go.numpy()},
             "grid": {"table": gg.numpy()}}
    return losses, grads
