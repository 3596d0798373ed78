"""The C-ABI library loads and exports every symbol include/aplicur.h declares
(CPU only: no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "aplicur.h")).read()
    return sorted(set(re.findall(r"\b(aplicur_[a-z_]+)\s*\(", text)))


def test_header_declares_the_four_entry_points():
    syms = declared_symbols()
    for name in ["aplicur_sketch", "aplicur_solve", "aplicur_solve_batched", "aplicur_solve_backward"]:
        assert name in syms


def test_library_exports_all_declared_symbols():
    from paper_2604_05065_amd import _lib
    lib = _lib.load()
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert set(_lib.EXPORTS) == set(declared_symbols())


def test_struct_layouts_match_header():
    from paper_2604_05065_amd import _lib
    # sizes fixed by the header's field lists (natural alignment, x86-64)
    assert ctypes.sizeof(_lib.Mat) == 4 + 4 + 8 * 4 + 8 * 3
    assert ctypes.sizeof(_lib.Opts) == 8 + 8 + 8 * 6 + 4 * 5 + 4 * 7 + 8 + 8  # tc_sketched + pad
    assert _lib.Opts.jacobi_tol.offset == 112 and _lib.Opts.tc_sketched.offset == 120
    assert ctypes.sizeof(_lib.Info) == 4 * 8 + 8 * 7
    assert _lib.Info.eta.offset == 32


def test_defaults_and_errors_without_gpu():
    from paper_2604_05065_amd import _lib
    lib = _lib.load()
    o = _lib.Opts()
    lib.aplicur_opts_default(ctypes.byref(o))
    assert (o.block, o.r_probes, o.nu_prec, o.nu_lsqr, o.eps_lsqr, o.tol_ne, o.precond) == \
        (20, 10, 10.0, 100.0, 1e-10, 1e-8, 1)
    # argument validation happens before any device work
    m = _lib.Mat(_lib.DENSE, _lib.F64, 10, 20, 20, 0, None, None, None)
    ctx = ctypes.c_void_p()
    assert lib.aplicur_sketch(ctypes.byref(m), ctypes.byref(o), None, 0, None, ctypes.byref(ctx)) == _lib.E_INVALID
    assert b"null" in lib.aplicur_last_error()
    m.val = 1  # non-null but mu = 0 with m < n is rejected before any device access
    assert lib.aplicur_sketch(ctypes.byref(m), ctypes.byref(o), None, 0, None, ctypes.byref(ctx)) == _lib.E_INVALID
    assert b"m >= n" in lib.aplicur_last_error()
    m2 = _lib.Mat(_lib.DENSE, _lib.F64, 20, 10, 10, 0, 1, None, None)
    o.precision = 3
    assert lib.aplicur_sketch(ctypes.byref(m2), ctypes.byref(o), None, 0, None, ctypes.byref(ctx)) == _lib.E_INVALID
    assert b"precision" in lib.aplicur_last_error()
    o.precision = 0
    # the SVD-free preconditioner is defined for mu = 0 only; precond is 0..2
    o.precond, o.mu = 2, 1e-4
    assert lib.aplicur_sketch(ctypes.byref(m2), ctypes.byref(o), None, 0, None, ctypes.byref(ctx)) == _lib.E_INVALID
    assert b"SVD-free" in lib.aplicur_last_error()
    o.precond, o.mu = 3, 0.0
    assert lib.aplicur_sketch(ctypes.byref(m2), ctypes.byref(o), None, 0, None, ctypes.byref(ctx)) == _lib.E_INVALID
    assert b"precond" in lib.aplicur_last_error()
    o.precond = 1
    assert lib.aplicur_ctx_query(None, 1, None, 0) == _lib.E_INVALID
    # workspace arguments are checked before any device access
    o.mu = 0.0
    assert lib.aplicur_sketch(ctypes.byref(m2), ctypes.byref(o), 4096, 0, None, ctypes.byref(ctx)) == _lib.E_INVALID
    assert b"ws_bytes" in lib.aplicur_last_error()
    assert lib.aplicur_sketch(ctypes.byref(m2), ctypes.byref(o), 4096 + 8, 1 << 20, None,
                              ctypes.byref(ctx)) == _lib.E_INVALID
    assert b"aligned" in lib.aplicur_last_error()
    assert lib.aplicur_workspace_bytes(ctypes.byref(m2), 0, ctypes.byref(o), None) == _lib.E_INVALID

def test_sketch_noalloc_rejects_what_does_not_fit():
    """aplicur_sketch_noalloc checks its scratch need on the host before any
    device access: 2^22 rows need 2^22 * 17 bytes for the sketch's rows and
    signs alone, more than its fixed 64 MiB (the values are never read)."""
    from paper_2604_05065_amd import _lib
    lib = _lib.load()
    o = _lib.Opts()
    lib.aplicur_opts_default(ctypes.byref(o))
    o.block = 100
    m = _lib.Mat(_lib.DENSE, _lib.F64, 1 << 22, 64, 64, 0, 256, None, None)
    assert lib.aplicur_sketch_noalloc(ctypes.byref(m), ctypes.byref(o), 4096, None) == _lib.E_INVALID
    assert b"bytes of scratch" in lib.aplicur_last_error()
    o.sketch = 1
    assert lib.aplicur_sketch_noalloc(ctypes.byref(m), ctypes.byref(o), 4096, None) == _lib.E_INVALID
    assert b"sparse sign" in lib.aplicur_last_error()


def test_product_timing_record_without_gpu():
    """aplicur_prof_read on an empty record returns zeros without device
    work, rejects null arrays, and switching timing off needs no device."""
    from paper_2604_05065_amd import _lib
    lib = _lib.load()
    n = 6
    cnt, tot, unt = (ctypes.c_int64 * n)(), (ctypes.c_double * n)(), (ctypes.c_int64 * n)()
    assert lib.aplicur_prof_products(0) == _lib.OK
    assert lib.aplicur_prof_read(cnt, tot, unt) == _lib.OK
    assert list(cnt) == [0] * n and list(tot) == [0.0] * n and list(unt) == [0] * n
    assert lib.aplicur_prof_read(None, tot, unt) == _lib.E_INVALID


def test_batched_workspace_arguments_checked_without_gpu():
    """aplicur_solve_batched rejects a misaligned workspace and
    aplicur_batched_workspace_bytes an empty batch before any device work."""
    from paper_2604_05065_amd import _lib
    lib = _lib.load()
    o = _lib.Opts()
    lib.aplicur_opts_default(ctypes.byref(o))
    m = (_lib.Mat * 1)(_lib.Mat(_lib.DENSE, _lib.F64, 20, 10, 10, 0, 1, None, None))
    ptrs = (ctypes.c_void_p * 1)(8)
    lds = (ctypes.c_int64 * 1)(20)
    infos = (_lib.Info * 1)()
    rc = lib.aplicur_solve_batched(1, m, ptrs, lds, 1, ptrs, lds, ctypes.byref(o), 4096 + 8, 1 << 20, infos, None)
    assert rc == _lib.E_INVALID and b"aligned" in lib.aplicur_last_error()
    assert lib.aplicur_batched_workspace_bytes(0, m, 1, ctypes.byref(o), None) == _lib.E_INVALID
