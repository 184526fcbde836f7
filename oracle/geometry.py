"""Ray-surfel geometry and the generalised-Gaussian kernel in FP64 (oracle).

Paper references:
  * Preliminaries, 2D Gaussian Splatting: a surfel has centre mu, rotation
    R = [v1, v2, v3] (v1, v2 span the surfel, v3 is its normal) and scales
    (s1, s2); a ray o + t d meets it at primitive-space coordinates (u, v).
  * Representation, Geometry: alpha = o * exp(-|u|^(2 g1) / 2) * exp(-|v|^(2 g2) / 2)
    with g >= 1; g = 1 gives the plain Gaussian of 2D Gaussian splatting.
  * Representation, Appearance: t* is the intersection depth and
    x* = o + t* d the world-space intersection.

All functions work on torch float64 tensors and are differentiable with
autograd; they broadcast, so the same code evaluates a [pixels, surfels]
grid or a flat list of pairs.
"""
from __future__ import annotations

import torch


def dot3(a, b):
    """(a0 b0 + a1 b1) + a2 b2 over the last axis, evaluated in that order."""
    return (a[..., 0] * b[..., 0] + a[..., 1] * b[..., 1]) + a[..., 2] * b[..., 2]


def quat_columns(q):
    """Columns v1, v2, v3 of the rotation of unit quaternion q = (w, x, y, z).

    The textbook unit-quaternion matrix, taking q as given.
    """
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    r00 = 1.0 - 2.0 * (y * y + z * z)
    r01 = 2.0 * (x * y - w * z)
    r02 = 2.0 * (x * z + w * y)
    r10 = 2.0 * (x * y + w * z)
    r11 = 1.0 - 2.0 * (x * x + z * z)
    r12 = 2.0 * (y * z - w * x)
    r20 = 2.0 * (x * z - w * y)
    r21 = 2.0 * (y * z + w * x)
    r22 = 1.0 - 2.0 * (x * x + y * y)
    v1 = torch.stack([r00, r10, r20], dim=-1)
    v2 = torch.stack([r01, r11, r21], dim=-1)
    v3 = torch.stack([r02, r12, r22], dim=-1)
    return v1, v2, v3


def camera_origin_and_rays(cam, px, py):
    """World-space camera centre o [3] and ray directions d [P,3].

    Pinhole model with the pixel centre at (px + 0.5, py + 0.5): the
    camera-frame direction is ((px+0.5-cx)/fx, (py+0.5-cy)/fy, 1), so the
    parameter t along o + t d is the camera-space depth.
    """
    m = torch.as_tensor(cam.world_to_cam, dtype=torch.float64)
    r = m[:, :3]
    tr = m[:, 3]
    px = torch.as_tensor(px, dtype=torch.float64)
    py = torch.as_tensor(py, dtype=torch.float64)
    dcx = (px + 0.5 - cam.cx) / cam.fx
    dcy = (py + 0.5 - cam.cy) / cam.fy
    dcz = torch.ones_like(dcx)
    d = torch.stack([(r[0, k] * dcx + r[1, k] * dcy) + r[2, k] * dcz for k in range(3)], dim=-1)
    o = -torch.stack([(r[0, k] * tr[0] + r[1, k] * tr[1]) + r[2, k] * tr[2] for k in range(3)])
    return o, d


def intersect(o, d, mu, v1, v2, v3, sig):
    """Ray-plane intersection of o + t d with the surfel plane.

    Returns (t, u, v, den): t = ((mu - o) . v3) / (d . v3), the hit point
    X = o + t d, u = ((X - mu) . v1) / s1 and v = ((X - mu) . v2) / s2.
    """
    den = dot3(d, v3)
    num = dot3(mu - o, v3)
    t = num / den
    X = o + t.unsqueeze(-1) * d
    q = X - mu
    u = dot3(q, v1) / sig[..., 0]
    v = dot3(q, v2) / sig[..., 1]
    return t, u, v, den


def abs_pow(a, e):
    """|a|^e for e >= 1, with the value 0 and a zero exponent-gradient at a = 0."""
    aa = a.abs()
    pos = aa > 0
    safe = torch.where(pos, aa, torch.ones_like(aa))
    return torch.where(pos, torch.exp(e * torch.log(safe)), torch.zeros_like(aa))


def kernel(u, v, gamma):
    """Generalised-Gaussian falloff exp(-|u|^(2 g1)/2 - |v|^(2 g2)/2)."""
    return torch.exp(-0.5 * abs_pow(u, 2.0 * gamma[..., 0]) - 0.5 * abs_pow(v, 2.0 * gamma[..., 1]))
