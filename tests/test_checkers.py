"""The parity tests' decision checker accepts exact decisions and rejects
planted wrong ones (CPU only; the "kernel" outputs here are built from the
oracle's own FP64 decisions)."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
import scenes
from oracle.mlp import hidden_preactivations
from tests.gpu_helpers import check_forced_decisions


@pytest.fixture(scope="module")
def case():
    wl = scenes.make_workload(1, seed=2, width=40, height=32)
    cam = wl.cameras[0]
    nat = oracle.render(wl.scene, cam, wl.grid, wl.mlp, wl.K, want_decisions=True)
    has = nat.ids >= 0
    cells = np.where(has[..., None, None], np.floor(np.nan_to_num(nat.lattice)), 0).astype(np.int64)
    z = nat.features
    W = [w.double().numpy() for w in wl.mlp.weights]
    H = W[0].shape[0]
    pre1, pre2 = hidden_preactivations(z.reshape(-1, z.shape[-1]), W)
    bits = np.concatenate([pre1 > 0, pre2 > 0], axis=1).reshape(-1, 2 * H // 32, 32).astype(np.uint64)
    words = (bits << np.arange(32, dtype=np.uint64)).sum(-1).astype(np.uint32).reshape(*z.shape[:2], -1)
    words = np.where(has[..., None], words, 0).astype(np.uint32)
    return wl, cam, nat, cells, words, z.astype(np.float32), nat.depths.astype(np.float32)


def test_exact_decisions_pass(case):
    wl, cam, nat, cells, words, feats, depths = case
    st = check_forced_decisions(nat, cells, words, feats, depths, cam, wl.grid.level_scales, wl.mlp.weights, "f32")
    assert st["slots"] > 1000 and st["cell_bad"] == 0 and st["relu_diff"] == 0


def test_wrong_cell_is_caught(case):
    wl, cam, nat, cells, words, feats, depths = case
    bad = cells.copy()
    dec = (nat.margin > 2.0)[:, None] & (nat.ids >= 0)
    p, j = np.argwhere(dec)[len(np.argwhere(dec)) // 2]
    lat = nat.lattice[p, j, 3]
    # move one coordinate a cell away from the face it is farthest from
    a = int(np.argmax(np.abs(lat - np.floor(lat) - 0.5) < 0.4))
    bad[p, j, 3, a] += 1 if lat[a] - np.floor(lat[a]) < 0.5 else -1
    with pytest.raises(AssertionError, match="hash cell"):
        check_forced_decisions(nat, bad, words, feats, depths, cam, wl.grid.level_scales, wl.mlp.weights, "f32")


def test_wrong_relu_bit_is_caught(case):
    wl, cam, nat, cells, words, feats, depths = case
    z = nat.features
    W = [w.double().numpy() for w in wl.mlp.weights]
    pre1, _ = hidden_preactivations(z.reshape(-1, z.shape[-1]), W)
    dec = ((nat.margin > 2.0)[:, None] & (nat.ids >= 0)).reshape(-1)
    # the decisive slot and unit with the largest |pre-activation| of layer 1
    mag = np.where(dec[:, None], np.abs(pre1), -1.0)
    s, u = np.unravel_index(np.argmax(mag), mag.shape)
    bad = words.copy().reshape(-1, words.shape[-1])
    bad[s, u // 32] ^= np.uint32(1 << (u % 32))
    with pytest.raises(AssertionError, match="ReLU layer 1"):
        check_forced_decisions(nat, cells, bad.reshape(words.shape), feats, depths, cam, wl.grid.level_scales,
                               wl.mlp.weights, "f32")


def test_feature_error_is_caught(case):
    wl, cam, nat, cells, words, feats, depths = case
    bad = feats.copy()
    p, j = np.argwhere((nat.margin > 2.0)[:, None] & (nat.ids >= 0))[0]
    bad[p, j, 0] += 1e-3
    with pytest.raises(AssertionError, match="feature error"):
        check_forced_decisions(nat, cells, words, bad, depths, cam, wl.grid.level_scales, wl.mlp.weights, "f32")
