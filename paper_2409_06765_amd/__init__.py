"""MI355X-native differentiable tile rasterizer for 3D Gaussian Splatting
(the rendering core of gsplat, arXiv 2409.06765).

The compute path is a HIP library for gfx950 (``libgsraster.so``) behind a
C ABI declared in ``include/gsraster.h``; ``_lib`` binds it with ctypes and
``rasterize`` wraps it in a ``torch.autograd.Function``.  Submodules load the
library lazily, so ``scenes`` (seeded synthetic inputs) imports without it.
"""

__all__ = ["rasterization", "load_library"]


def load_library():
    from . import _lib
    return _lib.lib()


def rasterization(*args, **kwargs):
    from .rasterize import rasterization as _r
    return _r(*args, **kwargs)
