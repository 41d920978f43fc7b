"""MI355X (gfx950) occupancy-grid ray marching and packed differentiable
volume rendering, after NerfAcc (Li, Tancik, Kanazawa, arXiv 2210.04847).

The compute runs in hand-written HIP kernels behind a C ABI (include/nacc.h);
PyTorch only supplies device memory and streams.  Importing the package
requires the built library (python paper_2210_04847_amd/build.py).
"""
from . import _lib
from ._lib import NaccError, version
from .api import (AttrsFn, BlobField, OccupancyGrid, RenderFn, STEP_1024, prune_samples,
                  ray_marching, render_attrs, render_fused, render_mse, rendering)

__all__ = ["AttrsFn", "BlobField", "NaccError", "OccupancyGrid", "RenderFn", "STEP_1024",
           "prune_samples", "ray_marching", "render_attrs", "render_fused", "render_mse",
           "rendering", "version", "_lib"]
