"""MI355X (gfx950) GMM superpixel EM: HIP kernels behind a C ABI (libgmmsp.so)
with a thin ctypes front end.  Importing the package loads nothing; the
library is loaded on first use and its absence is an error."""

__all__ = ["GMMSP", "grid", "make_params"]


def __getattr__(name):
    if name in __all__:
        from . import gmmsp
        return getattr(gmmsp, name)
    raise AttributeError(name)
