"""Numeric constants of the rendering method, as the oracle reads them.

The paper builds on the 3D Gaussian Splatting rasteriser and does not print
these values; each is a stated reading (see the design notes):
  ALPHA_MIN  an intersection whose alpha is below 1/255 is skipped.
  ALPHA_MAX  alpha is clamped to 0.99.
  T_MIN      compositing stops before the surfel that would take the
             transmittance below 1e-4; that surfel is not composited.
  SUPPORT    the kernel has a hard support |u| <= 3 and |v| <= 3.
  NEAR       camera-space depth of the near plane.
  TILE       screen tile edge in pixels for binning.
  MARGIN_PX  pixel margin added to each projected bounding box.
  PRIMES     spatial-hash multipliers of Instant-NGP (x, y, z).
"""

ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
T_MIN = 1e-4
SUPPORT = 3.0
NEAR = 0.2
TILE = 16
MARGIN_PX = 1.0
PRIMES = (1, 2654435761, 805459861)
