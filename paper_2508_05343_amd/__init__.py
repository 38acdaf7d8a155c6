"""MI355X (gfx950) 3D Gabor splatting rasterizer.

The compute path is libgabsplat.so (hand-written HIP kernels behind the C ABI
in include/gabsplat.h); this package holds its ctypes binding, a torch-facing
layer (device scenes, per-batch buffers, autograd) and the serving loop.
"""
from . import _lib  # noqa: F401
from ._lib import GabsplatError  # noqa: F401
