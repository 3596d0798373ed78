"""APLICUR on MI355X: adaptive CUR-preconditioned LSQR behind a C ABI.

The solver lives in libaplicur.so (hand-written gfx950 HIP kernels plus a
C++ driver, see include/aplicur.h); this package is its Python binding.
Importing it requires the built library -- there is no CPU fallback.
"""
from ._lib import AplicurError, load as _load
from .api import Context, CSRMatrix, lstsq, make_opts, sketch, solve_batched

_load()

__all__ = ["AplicurError", "Context", "CSRMatrix", "lstsq", "make_opts", "sketch", "solve_batched"]
