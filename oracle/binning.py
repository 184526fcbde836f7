"""Per-surfel preprocessing and tile binning in FP64 (oracle side).

Paper, Preliminaries (2D Gaussian Splatting): surfels are preprocessed and
sorted by the depth of their centres, then alpha-composited in a tile-based
rasteriser. The paper does not spell out the binning; this module states the
reading used here:

  * sort key: the camera-space z of the centre, rounded once to float32;
  * cull: non-finite inputs, a scale <= 0, or a centre at z <= NEAR;
  * footprint: the support rectangle mu +- 3 s1 v1 +- 3 s2 v2, clipped to
    z > NEAR (Sutherland-Hodgman against one plane), projected with the
    pinhole model; its bounding box widened by MARGIN_PX pixels selects the
    covered TILE x TILE screen tiles;
  * instances are ordered by (tile, key, surfel id).

Every FP64 expression below is evaluated in the order written, one rounding
per operation and no fused multiply-add (plain numpy float64 elementwise
arithmetic). The keys and tile lists are exact integer results of that
evaluation, so any other implementation that follows the same order obtains
the same bits.
"""
from __future__ import annotations

import numpy as np

from .constants import MARGIN_PX, NEAR, SUPPORT, TILE


def quat_columns_f64(q):
    """Rotation columns (v1, v2, v3) of the unit quaternion q = (w, x, y, z).

    The textbook unit-quaternion rotation matrix, taking q as given (the
    caller normalises). Each is an [N,3] float64 array.
    """
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    r00 = 1.0 - 2.0 * (y * y + z * z)
    r01 = 2.0 * (x * y - w * z)
    r02 = 2.0 * (x * z + w * y)
    r10 = 2.0 * (x * y + w * z)
    r11 = 1.0 - 2.0 * (x * x + z * z)
    r12 = 2.0 * (y * z - w * x)
    r20 = 2.0 * (x * z - w * y)
    r21 = 2.0 * (y * z + w * x)
    r22 = 1.0 - 2.0 * (x * x + y * y)
    v1 = np.stack([r00, r10, r20], axis=1)
    v2 = np.stack([r01, r11, r21], axis=1)
    v3 = np.stack([r02, r12, r22], axis=1)
    return v1, v2, v3


def to_camera_f64(m, p):
    """World point(s) p [...,3] to the camera frame with m = [R | t] (3x4)."""
    out = []
    for k in range(3):
        out.append(((m[k, 0] * p[..., 0] + m[k, 1] * p[..., 1]) + m[k, 2] * p[..., 2]) + m[k, 3])
    return np.stack(out, axis=-1)


def _finite_rows(*arrays):
    ok = None
    for a in arrays:
        a2 = a.reshape(a.shape[0], -1)
        f = np.all(np.isfinite(a2), axis=1)
        ok = f if ok is None else (ok & f)
    return ok


def surfel_keys_and_rects(scene, cam):
    """Per-surfel sort key, cull flag and tile rectangle.

    Returns a dict of numpy arrays:
      key    [N] float32   camera-space centre depth (rounded once)
      alive  [N] bool      not culled
      rect   [N,4] int64   tx0, ty0, tx1, ty1 (inclusive); empty if tx0 > tx1
      count  [N] int64     number of covered tiles
    """
    mu = scene.means.double().numpy()
    q = scene.quats.double().numpy()
    sg = scene.scales.double().numpy()
    op = scene.opacities.double().numpy()
    gm = scene.gammas.double().numpy()
    col = scene.colors.double().numpy()
    m = np.asarray(cam.world_to_cam, dtype=np.float64)
    n = mu.shape[0]
    ntx = (cam.width + TILE - 1) // TILE
    nty = (cam.height + TILE - 1) // TILE

    v1, v2, _ = quat_columns_f64(q)
    muc = to_camera_f64(m, mu)
    key = muc[:, 2].astype(np.float32)
    alive = _finite_rows(mu, q, sg, op.reshape(-1, 1), gm, col)
    alive &= (sg[:, 0] > 0.0) & (sg[:, 1] > 0.0)
    alive &= muc[:, 2] > NEAR

    r1 = SUPPORT * sg[:, 0]
    r2 = SUPPORT * sg[:, 1]
    signs = [(-1.0, -1.0), (1.0, -1.0), (1.0, 1.0), (-1.0, 1.0)]
    corners = []
    for a, b in signs:
        ra = a * r1
        rb = b * r2
        p = np.stack([(mu[:, k] + ra * v1[:, k]) + rb * v2[:, k] for k in range(3)], axis=1)
        corners.append(to_camera_f64(m, p))

    # Sutherland-Hodgman clip of the quad against z > NEAR.
    verts = np.zeros((n, 8, 3))
    vmask = np.zeros((n, 8), dtype=bool)
    slot = 0
    for i in range(4):
        A = corners[i]
        B = corners[(i + 1) % 4]
        ina = A[:, 2] > NEAR
        inb = B[:, 2] > NEAR
        verts[:, slot] = A
        vmask[:, slot] = ina
        slot += 1
        cross = ina != inb
        with np.errstate(divide="ignore", invalid="ignore"):
            s = (NEAR - A[:, 2]) / (B[:, 2] - A[:, 2])
            inter = np.stack([A[:, k] + s * (B[:, k] - A[:, k]) for k in range(3)], axis=1)
        verts[:, slot] = np.where(cross[:, None], inter, 0.0)
        vmask[:, slot] = cross
        slot += 1

    with np.errstate(divide="ignore", invalid="ignore"):
        X = cam.fx * (verts[..., 0] / verts[..., 2]) + cam.cx
        Y = cam.fy * (verts[..., 1] / verts[..., 2]) + cam.cy
    big = np.inf
    xmin = np.where(vmask, X, big).min(axis=1)
    xmax = np.where(vmask, X, -big).max(axis=1)
    ymin = np.where(vmask, Y, big).min(axis=1)
    ymax = np.where(vmask, Y, -big).max(axis=1)
    has = vmask.any(axis=1)
    alive &= has

    with np.errstate(invalid="ignore"):
        tx0 = np.floor((xmin - MARGIN_PX) / TILE)
        tx1 = np.floor((xmax + MARGIN_PX) / TILE)
        ty0 = np.floor((ymin - MARGIN_PX) / TILE)
        ty1 = np.floor((ymax + MARGIN_PX) / TILE)
    tx0 = np.clip(np.nan_to_num(tx0, nan=1e18), 0.0, float(ntx)).astype(np.int64)
    tx1 = np.clip(np.nan_to_num(tx1, nan=-1e18), -1.0, float(ntx - 1)).astype(np.int64)
    ty0 = np.clip(np.nan_to_num(ty0, nan=1e18), 0.0, float(nty)).astype(np.int64)
    ty1 = np.clip(np.nan_to_num(ty1, nan=-1e18), -1.0, float(nty - 1)).astype(np.int64)
    nonempty = (tx0 <= tx1) & (ty0 <= ty1) & alive
    count = np.where(nonempty, (tx1 - tx0 + 1) * (ty1 - ty0 + 1), 0)
    rect = np.stack([tx0, ty0, tx1, ty1], axis=1)
    return {"key": key, "alive": alive, "rect": rect, "count": count, "ntx": ntx, "nty": nty}


def bin_surfels(scene, cam):
    """Tile instances sorted by (tile, key, id) and per-tile [start, end).

    Returns a dict with
      tiles  [I] int64, ids [I] int64, keys [I] float32   (sorted order)
      ranges [n_tiles, 2] int64
      plus everything from surfel_keys_and_rects.
    """
    info = surfel_keys_and_rects(scene, cam)
    ntx, nty = info["ntx"], info["nty"]
    rect, count, key = info["rect"], info["count"], info["key"]
    sel = np.nonzero(count > 0)[0]
    cnt = count[sel]
    ids = np.repeat(sel, cnt)
    first = np.repeat(np.cumsum(cnt) - cnt, cnt)
    local = np.arange(ids.shape[0], dtype=np.int64) - first
    width = rect[ids, 2] - rect[ids, 0] + 1
    tiles = (rect[ids, 1] + local // width) * ntx + (rect[ids, 0] + local % width)
    keys = key[ids]
    order = np.lexsort((ids, keys, tiles))
    tiles, ids, keys = tiles[order], ids[order], keys[order]
    n_tiles = ntx * nty
    starts = np.searchsorted(tiles, np.arange(n_tiles), side="left")
    ends = np.searchsorted(tiles, np.arange(n_tiles), side="right")
    info.update({"tiles": tiles, "ids": ids, "keys": keys, "ranges": np.stack([starts, ends], axis=1)})
    return info
