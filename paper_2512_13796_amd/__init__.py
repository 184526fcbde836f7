"""MI355X (gfx950) implementation of the Nexels rendering path.

Importing the package loads libnexels.so (built by
``python paper_2512_13796_amd/build.py``) and raises ImportError if it is
missing: there is no CPU or eager-PyTorch fallback.
"""
from . import _lib

_lib.load()

from .render import (Context, ForwardResult, RenderFunction, autotune_raster, aux_losses,  # noqa: E402,F401
                     camera_struct, densify, fps, instance_counts, render, render_backward, render_forward,
                     render_forward_noalloc, workspace_size, workspace_size_exact)

__all__ = ["Context", "ForwardResult", "RenderFunction", "autotune_raster", "aux_losses", "camera_struct", "densify",
           "fps", "instance_counts", "render", "render_backward", "render_forward", "render_forward_noalloc",
           "workspace_size", "workspace_size_exact"]
