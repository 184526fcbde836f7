"""Multiresolution hash-grid encoding with down-weighting, FP64 (oracle).

Paper references:
  * Preliminaries, Instant-NGP: L levels, each a table of T entries with F
    features, queried at s_l * x; the per-level features are concatenated.
  * Supplementary, Implementation Details, Architecture: a hash is used at
    every level (no dense coarse levels), inputs are unbounded, and the
    integer lattice coordinates go through MapPositive before hashing:
    MapPositive(z) = 2z - 1 for z > 0 and -2z otherwise.
  * Supplementary, Other details: features are interpolated trilinearly
    and the sample position receives a gradient through the interpolation.
  * eq. downweighting: level l is scaled by
    Delta_l = 1 - exp(-(f / (s_l t*))^2 / (2 pi)).

The spatial hash is Instant-NGP's: XOR of the coordinates times the primes
(1, 2654435761, 805459861), modulo 2^32, then masked to the table size.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .constants import PRIMES


def map_positive(z):
    """MapPositive on int64 numpy arrays: a bijection from Z onto N."""
    z = np.asarray(z, dtype=np.int64)
    return np.where(z > 0, 2 * z - 1, -2 * z)


def spatial_hash(kx, ky, kz, log2_size):
    """Instant-NGP spatial hash of non-negative lattice coordinates."""
    mask32 = np.uint64(0xFFFFFFFF)
    ux = np.asarray(kx).astype(np.uint64) & mask32
    uy = np.asarray(ky).astype(np.uint64) & mask32
    uz = np.asarray(kz).astype(np.uint64) & mask32
    with np.errstate(over="ignore"):
        h = (ux * np.uint64(PRIMES[0])) ^ (uy * np.uint64(PRIMES[1])) ^ (uz * np.uint64(PRIMES[2]))
    h = h & mask32
    return (h & np.uint64((1 << log2_size) - 1)).astype(np.int64)


def downweight(depth, level_scale, focal):
    """Delta = 1 - exp(-(f / (s t))^2 / (2 pi)), evaluated as -expm1(-y)."""
    y = (focal / (level_scale * depth)) ** 2 / (2.0 * math.pi)
    return -torch.expm1(-y)


def encode(x, depth, table, level_scales, focal, cells=None):
    """Concatenation over levels of Delta_l * H_l(s_l x), shape [S, L*F].

    x [S,3] and depth [S] are float64 (differentiable); table [L,T,F] float64.
    Per level: p = s_l x, c0 = floor(p), fr = p - c0; each of the 8 cell
    corners c0 + b is hashed after MapPositive and weighted by
    prod_axis (b ? fr : 1 - fr).

    cells [S,L,3] (optional, int) replaces floor(p) by a given lattice cell:
    the same trilinear polynomial of that cell is evaluated at p (fr may
    leave [0,1] by a rounding-sized amount). Used to evaluate a sample under
    the cell decision another implementation took.
    """
    L, Tsz, F = table.shape
    log2_size = int(Tsz).bit_length() - 1
    S = x.shape[0]
    idx = np.zeros((S, L, 8), dtype=np.int64)
    wts = []
    for l in range(L):
        p = float(level_scales[l]) * x
        if cells is None:
            c0 = torch.floor(p).detach()
        else:
            c0 = torch.as_tensor(np.asarray(cells)[:, l, :], dtype=torch.float64)
        fr = p - c0
        c0i = c0.numpy().astype(np.int64)
        wl = []
        for corner in range(8):
            b = [(corner >> a) & 1 for a in range(3)]
            k = [map_positive(c0i[:, a] + b[a]) for a in range(3)]
            idx[:, l, corner] = l * Tsz + spatial_hash(k[0], k[1], k[2], log2_size)
            w = None
            for a in range(3):
                wa = fr[:, a] if b[a] else 1.0 - fr[:, a]
                w = wa if w is None else w * wa
            wl.append(w)
        wts.append(torch.stack(wl, dim=1))
    vals = table.reshape(L * Tsz, F)[torch.from_numpy(idx.reshape(-1))].reshape(S, L, 8, F)
    feats = []
    for l in range(L):
        f = (wts[l].unsqueeze(-1) * vals[:, l]).sum(dim=1)
        feats.append(downweight(depth, float(level_scales[l]), focal).unsqueeze(1) * f)
    return torch.cat(feats, dim=1)
