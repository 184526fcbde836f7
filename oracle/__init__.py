"""Plain, slow FP64 CPU oracle for the Nexels rendering path.

TEST INFRASTRUCTURE ONLY. Nothing in the product package imports this
package; only the tests, the smoke check and the benchmark's CPU-baseline
leg may call it. It shares no code with the HIP path: the only common input
is the seeded scene generator (``scenes``), which holds no rendering
arithmetic.

What it computes (paper: Nexels, arXiv 2512.13796):
  * binning.py   per-surfel centre depth, sort key and screen tile rectangle
                 (Preliminaries, 2D Gaussian Splatting: surfels are
                 preprocessed and sorted by the depth of their centres and
                 composited in a tile-based rasteriser).
  * geometry.py  quaternion rotation, pinhole rays, ray-surfel intersection
                 (u, v, t*) and the generalised-Gaussian kernel
                 (Representation, Geometry).
  * hashgrid.py  MapPositive, spatial hash, trilinear hash-grid encoding and
                 the anti-aliasing down-weighting (Preliminaries, Instant-NGP;
                 eq. downweighting; supplementary Implementation Details).
  * mlp.py       bias-free ReLU MLP with a sigmoid head (Results,
                 implementation details; supplementary Anti-aliasing).
  * sh.py        degree-3 real spherical harmonics and the view-dependent
                 colour decode (Representation, Appearance).
  * losses.py    the auxiliary losses L_alpha, L_texture, L_opacity, L_grid and
                 their gradients (Optimization, Losses).
  * adc.py       farthest point sampling, error-weighted split selection, the
                 split geometry and pruning (supplementary, Adaptive Density
                 Control).
  * render.py    collection pass (eq. composite, eq. notexture, K-buffer by
                 weight), texturing pass (eq. texture) and the final
                 composite (eq. final), untiled, with a per-pixel brute-force
                 loop over every surfel; gradients by reverse-mode autograd
                 through the same FP64 expressions with every discrete
                 decision held fixed.

Pins (tests/test_oracle_pins.py) tie each function to closed forms,
invariants, limits and finite differences rather than to itself.
"""

from .render import OracleOutputs, render, render_and_grad  # noqa: F401
from .binning import bin_surfels  # noqa: F401
