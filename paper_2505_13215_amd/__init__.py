"""MI355X-native hybrid 3D/4D Gaussian rasterizer.

The HIP library ``libh4dgs.so`` (C ABI in ``include/h4dgs.h``) does all of
the work; ``render.py`` binds it to PyTorch tensors and autograd.
"""
from . import _lib
from ._lib import H4DError, version
from .autotune import CANDIDATES, Autotuner
from .render import (CapturedStep, DEFAULT_CHUNK, DEFAULT_TILE, G3_KEYS, G4_KEYS, H4DGSRender, Rasterizer, adam_step, convert_static, l1_loss_grad,
                     rasterize_splats, render, render_infer_noalloc, to_device, densify, new_stats)

__all__ = ["H4DError", "version", "Autotuner", "CANDIDATES", "CapturedStep", "DEFAULT_TILE", "DEFAULT_CHUNK", "G3_KEYS", "G4_KEYS", "H4DGSRender", "Rasterizer", "adam_step", "convert_static",
           "rasterize_splats", "render", "render_infer_noalloc", "to_device", "densify", "new_stats", "l1_loss_grad", "_lib"]
