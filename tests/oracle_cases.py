"""Small hand-built scenes for the oracle pins (no rendering arithmetic here)."""
from __future__ import annotations

import numpy as np
import torch

from scenes import MLP, Camera, HashGrid, Scene


def identity_camera(width=32, height=32, focal=40.0):
    m = np.zeros((3, 4))
    m[:, :3] = np.eye(3)
    return Camera(m, focal, focal, width / 2.0, height / 2.0, width, height)


def scene_from(means, quats, scales, opac, gammas, colors, dtype=torch.float64):
    f = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float64), dtype=dtype)
    return Scene(f(means), f(quats), f(scales), f(opac), f(gammas), f(colors))


def constant_grid(values_per_level, log2_size=8, scales=(16.0, 24.0)):
    """Grid whose every entry at level l equals values_per_level[l] (F values)."""
    vals = np.asarray(values_per_level, dtype=np.float64)
    L, F = vals.shape
    table = np.broadcast_to(vals[:, None, :], (L, 1 << log2_size, F)).copy()
    return HashGrid(torch.from_numpy(table), torch.tensor(scales[:L], dtype=torch.float32))


def random_grid(rng, levels=2, log2_size=8, feat=2, scale=0.5):
    table = rng.uniform(-scale, scale, (levels, 1 << log2_size, feat))
    scales = (16.0 * 1.5 ** np.arange(levels)).astype(np.float32)
    return HashGrid(torch.from_numpy(table), torch.from_numpy(scales))


def random_mlp(rng, dims):
    ws = []
    for i in range(len(dims) - 1):
        b = np.sqrt(6.0 / (dims[i] + dims[i + 1]))
        ws.append(torch.from_numpy(rng.uniform(-b, b, (dims[i + 1], dims[i]))))
    return MLP(ws)


def facing_scene(rng, n, depth_range=(1.5, 3.0), xy=0.6, sigma=(0.05, 0.25), tilt=0.0):
    """n surfels in front of an identity camera; tilt > 0 randomises orientation."""
    z = rng.uniform(*depth_range, n)
    means = np.stack([rng.uniform(-xy, xy, n) * z / 2.0, rng.uniform(-xy, xy, n) * z / 2.0, z], axis=1)
    q = np.zeros((n, 4))
    q[:, 0] = 1.0
    q[:, 1:] = tilt * rng.standard_normal((n, 3))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    scales = rng.uniform(sigma[0], sigma[1], (n, 2))
    opac = rng.uniform(0.3, 0.95, n)
    gammas = np.ones((n, 2))
    colors = rng.uniform(0.0, 1.0, (n, 3))
    return scene_from(means, q, scales, opac, gammas, colors)
