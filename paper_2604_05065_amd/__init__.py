"""APLICUR on MI355X: adaptive CUR-preconditioned LSQR behind a C ABI.

The solver lives in libaplicur.so (hand-written gfx950 HIP kernels plus a
C++ driver, see include/aplicur.h); this package is its Python binding.
Every entry point loads the built library and fails loudly if it is missing
-- there is no CPU fallback.
"""
from ._lib import AplicurError, load as load_library
from .api import (Context, CSRMatrix, LstsqFunction, batched_workspace_bytes, lstsq, lstsq_autograd, make_opts,
                  prof_products, prof_read, sketch, sketch_noalloc, solve_batched, workspace_bytes)

__all__ = ["AplicurError", "load_library", "Context", "CSRMatrix", "LstsqFunction", "batched_workspace_bytes", "lstsq", "lstsq_autograd",
           "make_opts", "prof_products", "prof_read", "sketch", "sketch_noalloc", "solve_batched", "workspace_bytes"]
