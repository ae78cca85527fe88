"""Boundary Value Caching for walk on spheres on MI355X (gfx950).

The compute path is libbvc.so (HIP kernels behind a C-ABI, ``include/bvc.h``);
``_bvc`` binds it with ctypes and ``pipeline`` sequences the calls of
Algorithm 1.  Importing the package fails when the library is not built.
"""
from . import _bvc  # noqa: F401  (raises ImportError when libbvc.so is missing)
from . import pipeline  # noqa: F401

__all__ = ["_bvc", "pipeline"]
