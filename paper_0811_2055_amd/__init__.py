"""MI355X-native octree level-of-detail build and point splat.

The hot path runs in liblod.so (HIP kernels for gfx950, C ABI in
include/lod.h); this package binds it (``lib``) and adds the differentiable
splat (``autograd``) and the per-node refinement loop (``refine``).
"""
from . import lib  # noqa: F401

__all__ = ["lib"]
