"""MI355X-native latent Gaussian rasterizer (Tele-Aloha, arXiv 2405.14866, §4.2).

The hot path -- projection, tile binning and sort, front-to-back blend, and
its adjoint -- is hand-written HIP for gfx950 in ``libtg.so`` behind the C
ABI of ``include/tg.h``.  ``_native`` binds that ABI with ctypes;
``rasterize`` adds torch device memory, streams and autograd.
"""
from . import _native
from ._native import TgError

__all__ = ["_native", "TgError", "rasterize", "Rasterizer", "GaussianSoA", "Context", "Frame"]


def __getattr__(name):
    if name in ("rasterize", "Rasterizer", "GaussianSoA", "Context", "Frame", "camera_struct"):
        from . import rasterize as _r
        return getattr(_r, name)
    raise AttributeError(name)
