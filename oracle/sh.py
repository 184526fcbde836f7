"""View-dependent colour from real spherical harmonics (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper, Preliminaries (2D Gaussian Splatting) and Representation, Appearance:
each surfel's non-textured radiance is a set of channel-wise spherical
harmonics coefficients (degree 3: S = 16 per channel, 48 values), and the
neural field outputs the same number of coefficients for the textured
appearance (Results: the experiments use degree 3, hence 48 MLP outputs).

Readings (the paper builds on the 3D Gaussian Splatting code and does not
print these):
  * the real SH basis up to degree 3 in the usual Cartesian form, with the
    orthonormal constants below and the sign convention of that codebase;
  * coefficient layout [S][3]: coefficient k of channel c at index 3 k + c;
  * colour = max(0, sum_k Y_k(d) a_k + 0.5) per channel, so zero coefficients
    give grey 0.5 (the paper notes the texture is mostly grey where the
    field outputs little);
  * d is the unit direction from the camera centre to the surfel centre for
    the plain colour, and the unit ray direction of the pixel for the
    texture.
"""
from __future__ import annotations

import math

import torch

C0 = 0.5 / math.sqrt(math.pi)
C1 = math.sqrt(3.0 / (4.0 * math.pi))
C2 = (0.5 * math.sqrt(15.0 / math.pi), -0.5 * math.sqrt(15.0 / math.pi), 0.25 * math.sqrt(5.0 / math.pi),
      -0.5 * math.sqrt(15.0 / math.pi), 0.25 * math.sqrt(15.0 / math.pi))
C3 = (-0.25 * math.sqrt(35.0 / (2.0 * math.pi)), 0.5 * math.sqrt(105.0 / math.pi),
      -0.25 * math.sqrt(21.0 / (2.0 * math.pi)), 0.25 * math.sqrt(7.0 / math.pi),
      -0.25 * math.sqrt(21.0 / (2.0 * math.pi)), 0.25 * math.sqrt(105.0 / math.pi),
      -0.25 * math.sqrt(35.0 / (2.0 * math.pi)))


def basis(d, degree=3):
    """Y_k(d) for k < (degree + 1)^2 over the last axis of unit directions d [..., 3] -> [..., S]."""
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    out = [torch.full_like(x, C0)]
    if degree >= 1:
        out += [-C1 * y, C1 * z, -C1 * x]
    if degree >= 2:
        xx, yy, zz = x * x, y * y, z * z
        out += [C2[0] * x * y, C2[1] * y * z, C2[2] * (2.0 * zz - xx - yy), C2[3] * x * z, C2[4] * (xx - yy)]
    if degree >= 3:
        out += [C3[0] * y * (3.0 * xx - yy), C3[1] * x * y * z, C3[2] * y * (4.0 * zz - xx - yy),
                C3[3] * z * (2.0 * zz - 3.0 * xx - 3.0 * yy), C3[4] * x * (4.0 * zz - xx - yy),
                C3[5] * z * (xx - yy), C3[6] * x * (xx - 3.0 * yy)]
    return torch.stack(out, dim=-1)


def colour(coeffs, d, degree=3):
    """max(0, sum_k Y_k(d) a_{k,c} + 0.5): coeffs [..., S*3] in the [S][3] layout, d [..., 3] unit."""
    S = (degree + 1) ** 2
    a = coeffs.reshape(coeffs.shape[:-1] + (S, 3))
    y = basis(d, degree)
    return torch.clamp((y[..., :, None] * a).sum(dim=-2) + 0.5, min=0.0)
