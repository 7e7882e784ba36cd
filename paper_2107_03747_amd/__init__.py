"""Twisted Wilson flow on MI355X (gfx950).

``paper_2107_03747_amd.gen`` (seeded input fields) imports without the GPU
library.  Everything else is the thin ctypes binding of ``libtgf.so``
(``paper_2107_03747_amd.tgf``), imported on first use; it raises if the
library has not been built.
"""

__all__ = ["gen", "tgf"]


def __getattr__(name):
    if name in ("gen", "tgf", "build"):
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    from . import tgf as _tgf
    if hasattr(_tgf, name):
        return getattr(_tgf, name)
    raise AttributeError(name)
