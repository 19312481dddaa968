"""MI355X-native matrix-free DG residual, Jacobian-vector product, element
block-Jacobi preconditioner and flexible GMRES (HIP for gfx950).

The numerical work lives in libdg.so (C ABI in include/dg.h); `DG` is a thin
torch wrapper.  Importing `DG` requires the library to be built.
"""
from . import _lib  # noqa: F401


def __getattr__(name):
    if name == "DG":
        from .api import DG
        return DG
    raise AttributeError(name)
