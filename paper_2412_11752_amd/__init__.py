"""MI355X-native tile-based differentiable rasterizer for Deformable Radial Kernel (DRK) primitives.

The compute path is the HIP library libdrk.so (C ABI in include/drk.h); this package is a thin
torch binding around it.  Importing the package does not load the library; the first call does,
and fails loudly if it has not been built.
"""
from .rasterizer import (  # noqa: F401
    DRKScene, Rasterizer, DRKRenderFunction, render, camera_struct, make_opts, EXPORT, KEY_MODES, trace_metrics,
    mesh_to_drk, activate, activate_bwd, adam_step,
)

__all__ = ["DRKScene", "Rasterizer", "DRKRenderFunction", "render", "camera_struct", "make_opts", "EXPORT",
           "KEY_MODES", "trace_metrics", "mesh_to_drk", "activate", "activate_bwd", "adam_step"]
