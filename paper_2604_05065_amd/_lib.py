"""ctypes declarations of libaplicur.so (mirror of include/aplicur.h).

The library is loaded from this package directory only; if it is missing the
import fails loudly -- there is no CPU fallback.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaplicur.so")

OK, W_MAXITER, E_INVALID, E_HIP, E_BREAKDOWN, E_NOMEM = 0, 1, -1, -3, -4, -5
DENSE, DENSE_COL, CSR = 0, 1, 2
F64, F32 = 0, 1


class Mat(C.Structure):
    _fields_ = [("format", C.c_int32), ("dtype", C.c_int32), ("m", C.c_int64), ("n", C.c_int64),
                ("ld", C.c_int64), ("nnz", C.c_int64), ("val", C.c_void_p),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p)]


class Opts(C.Structure):
    _fields_ = [("block", C.c_int32), ("r_probes", C.c_int32), ("seed", C.c_uint64), ("mu", C.c_double),
                ("eps_cur", C.c_double), ("nu_prec", C.c_double), ("nu_lsqr", C.c_double),
                ("eps_lsqr", C.c_double), ("tol_ne", C.c_double), ("max_iter", C.c_int32),
                ("max_rank", C.c_int32), ("precond", C.c_int32), ("precision", C.c_int32),
                ("max_outer", C.c_int32), ("workers", C.c_int32), ("tune", C.c_int32),
                ("graphs", C.c_int32), ("columns", C.c_int32), ("xi", C.c_int32),
                ("sketch", C.c_int32), ("schedule", C.c_int32), ("jacobi_tol", C.c_double),
                ("tc_sketched", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("status", C.c_int32), ("phases", C.c_int32), ("iters", C.c_int32), ("rank", C.c_int32),
                ("rebuilds", C.c_int32), ("outer", C.c_int32), ("phases_bf16", C.c_int32),
                ("reserved", C.c_int32), ("eta", C.c_double), ("rho", C.c_double),
                ("sigma_hat", C.c_double), ("t_sketch_ms", C.c_double), ("t_cur_ms", C.c_double),
                ("t_precond_ms", C.c_double), ("t_lsqr_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = ["aplicur_opts_default", "aplicur_workspace_bytes", "aplicur_sketch", "aplicur_sketch_noalloc", "aplicur_solve", "aplicur_solve_batched", "aplicur_batched_workspace_bytes",
           "aplicur_solve_backward", "aplicur_matvec", "aplicur_matmat", "aplicur_time_product", "aplicur_time_matmat", "aplicur_precond_apply", "aplicur_ctx_query", "aplicur_ctx_destroy",
           "aplicur_prof_products", "aplicur_prof_read", "aplicur_last_error", "aplicur_version"]

_lib = None


def load():
    """Load libaplicur.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2604_05065_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.c_void_p
    lib.aplicur_opts_default.argtypes = [C.POINTER(Opts)]
    lib.aplicur_opts_default.restype = None
    lib.aplicur_sketch.argtypes = [C.POINTER(Mat), C.POINTER(Opts), vp, C.c_size_t, vp, C.POINTER(vp)]
    lib.aplicur_sketch.restype = C.c_int
    lib.aplicur_sketch_noalloc.argtypes = [C.POINTER(Mat), C.POINTER(Opts), dp, vp]
    lib.aplicur_sketch_noalloc.restype = C.c_int
    lib.aplicur_workspace_bytes.argtypes = [C.POINTER(Mat), i32, C.POINTER(Opts), vp]
    lib.aplicur_workspace_bytes.restype = C.c_int64
    lib.aplicur_solve.argtypes = [vp, dp, i64, i32, dp, i64, i32, C.POINTER(Info), vp]
    lib.aplicur_solve.restype = C.c_int
    lib.aplicur_solve_batched.argtypes = [i32, C.POINTER(Mat), C.POINTER(vp), C.POINTER(i64), i32,
                                          C.POINTER(vp), C.POINTER(i64), C.POINTER(Opts), vp, C.c_size_t,
                                          C.POINTER(Info), vp]
    lib.aplicur_batched_workspace_bytes.argtypes = [i32, C.POINTER(Mat), i32, C.POINTER(Opts), vp]
    lib.aplicur_batched_workspace_bytes.restype = C.c_int64
    lib.aplicur_solve_batched.restype = C.c_int
    lib.aplicur_solve_backward.argtypes = [vp, dp, i64, dp, i64, dp, i64, i32, dp, i64, dp, i64, dp, i64,
                                           C.POINTER(Info), vp]
    lib.aplicur_solve_backward.restype = C.c_int
    lib.aplicur_matvec.argtypes = [vp, i32, dp, dp, vp]
    lib.aplicur_matvec.restype = C.c_int
    lib.aplicur_matmat.argtypes = [vp, i32, dp, i64, i32, dp, i64, i32, vp]
    lib.aplicur_matmat.restype = C.c_int
    lib.aplicur_time_matmat.argtypes = [vp, i32, dp, i64, i32, dp, i64, i32, i32, vp, i64, vp, C.POINTER(C.c_double)]
    lib.aplicur_time_matmat.restype = C.c_int
    lib.aplicur_precond_apply.argtypes = [vp, i32, dp, dp, vp]
    lib.aplicur_precond_apply.restype = C.c_int
    lib.aplicur_time_product.argtypes = [vp, i32, dp, dp, i32, vp, i64, vp, C.POINTER(C.c_double)]
    lib.aplicur_time_product.restype = C.c_int
    lib.aplicur_prof_products.argtypes = [i32]
    lib.aplicur_prof_products.restype = C.c_int
    lib.aplicur_prof_read.argtypes = [C.POINTER(i64), C.POINTER(C.c_double), C.POINTER(i64)]
    lib.aplicur_prof_read.restype = C.c_int
    lib.aplicur_ctx_query.argtypes = [vp, i32, vp, C.c_size_t]
    lib.aplicur_ctx_query.restype = i64
    lib.aplicur_ctx_destroy.argtypes = [vp]
    lib.aplicur_ctx_destroy.restype = None
    lib.aplicur_last_error.argtypes = []
    lib.aplicur_last_error.restype = C.c_char_p
    lib.aplicur_version.argtypes = []
    lib.aplicur_version.restype = C.c_char_p
    _lib = lib
    return lib


class AplicurError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"aplicur error {code}: {msg}")
        self.code = code


def check(code):
    if code < 0:
        raise AplicurError(code, load().aplicur_last_error().decode(errors="replace"))
    return code
