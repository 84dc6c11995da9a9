"""MI355X-native 3DGUT rasterizer: Unscented-Transform projection, tile
binning by device radix sort, per-tile 3D-response compositing and its
backward, as hand-written HIP kernels for gfx950 behind the C ABI of
include/gut.h, plus a continuous-batching server.

The compute lives in ``libgut.so`` (built in-tree by ``build.py``); the
Python modules only marshal arguments.
"""
from . import _lib  # noqa: F401

__all__ = ["raster", "serve", "build"]
