"""Python binding of libaplicur.so (argument marshalling only).

Every step of the solve runs in the HIP library; PyTorch supplies device
memory and the current stream.  Inputs may be FP32 or FP64 for A; right-hand
sides and solutions are FP64.
"""
import ctypes as C
import math

import numpy as np
import torch

from . import _lib as L


class CSRMatrix:
    """A CSR matrix on the GPU: row_ptr (m+1, int32), col_idx (nnz, int32), val (nnz)."""

    def __init__(self, row_ptr, col_idx, val, shape):
        self.row_ptr = row_ptr.to(torch.int32).contiguous()
        self.col_idx = col_idx.to(torch.int32).contiguous()
        self.val = val.contiguous()
        self.shape = tuple(int(s) for s in shape)

    @classmethod
    def from_scipy(cls, A, device="cuda", dtype=torch.float64):
        A = A.tocsr()
        return cls(torch.as_tensor(A.indptr, device=device), torch.as_tensor(A.indices, device=device),
                   torch.as_tensor(A.data, device=device, dtype=dtype), A.shape)

    @property
    def dtype(self):
        return self.val.dtype


def _dtype_code(dt):
    if dt == torch.float64:
        return L.F64
    if dt == torch.float32:
        return L.F32
    raise TypeError(f"A must be float32 or float64, got {dt}")


def _mat(A):
    if isinstance(A, CSRMatrix):
        m, n = A.shape
        if not A.val.is_cuda:
            raise ValueError("A must live on the GPU")
        st = L.Mat(L.CSR, _dtype_code(A.val.dtype), m, n, 0, A.val.numel(), A.val.data_ptr(),
                   A.row_ptr.data_ptr(), A.col_idx.data_ptr())
        return st, (A.row_ptr, A.col_idx, A.val)
    if isinstance(A, torch.Tensor) and A.layout == torch.sparse_csr:
        return _mat(CSRMatrix(A.crow_indices(), A.col_indices(), A.values(), A.shape))
    if not isinstance(A, torch.Tensor) or A.dim() != 2:
        raise TypeError("A must be a 2-D torch tensor or a CSRMatrix")
    if not A.is_cuda:
        raise ValueError("A must live on the GPU")
    m, n = A.shape
    if A.stride(0) == 1 and A.stride(1) >= max(m, 1) and n > 1:  # column-major (e.g. a transposed view)
        st = L.Mat(L.DENSE_COL, _dtype_code(A.dtype), m, n, A.stride(1), 0, A.data_ptr(), None, None)
        return st, (A,)
    if A.stride(1) != 1:
        A = A.contiguous()
    st = L.Mat(L.DENSE, _dtype_code(A.dtype), m, n, A.stride(0), 0, A.data_ptr(), None, None)
    return st, (A,)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _device(A):
    return A.val.device if isinstance(A, CSRMatrix) else A.device


def make_opts(mu=0.0, block=20, seed=7, eps_cur=-1.0, nu_prec=10.0, nu_lsqr=100.0, eps_lsqr=1e-10,
              tol_ne=1e-8, max_iter=100000, max_rank=0, precond=True, precision=0, max_outer=0,
              r_probes=10, workers=0, tune=0, graphs=0, columns=0, xi=8, sketch=0, schedule=0,
              jacobi_tol=0.0, tc_sketched=False):
    lib = L.load()
    o = L.Opts()
    lib.aplicur_opts_default(C.byref(o))
    o.mu, o.block, o.seed, o.eps_cur = float(mu), int(block), int(seed), float(eps_cur)
    o.nu_prec, o.nu_lsqr, o.eps_lsqr, o.tol_ne = float(nu_prec), float(nu_lsqr), float(eps_lsqr), float(tol_ne)
    # precond: True / "svd" (APLICUR), "svdfree" (Alg. 8, mu = 0), False (plain LSQR)
    if isinstance(precond, str):
        precond = {"svd": 1, "svdfree": 2}[precond]
    o.max_iter, o.max_rank, o.precond = int(max_iter), int(max_rank), int(precond)
    o.precision, o.max_outer, o.r_probes = int(precision), int(max_outer), int(r_probes)
    o.workers, o.tune, o.graphs = int(workers), int(bool(tune)), int(bool(graphs))
    o.columns = int(bool(columns))
    o.xi = int(xi)
    o.sketch = {"sparse": 0, "gaussian": 1, "gaussian_bf16": 2}[sketch] if isinstance(sketch, str) else int(sketch)
    o.schedule = int(schedule)
    o.jacobi_tol = float(jacobi_tol)
    o.tc_sketched = int(bool(tc_sketched))
    return o


def _cols(B, rows, name):
    """FP64 column-major view of B (rows,) or (rows, k): returns (tensor (k, rows), k, was_1d)."""
    if not isinstance(B, torch.Tensor) or not B.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    one = B.dim() == 1
    Bm = B.reshape(rows, 1) if one else B
    if Bm.shape[0] != rows:
        raise ValueError(f"{name} has {Bm.shape[0]} rows, expected {rows}")
    return Bm.to(torch.float64).t().contiguous(), Bm.shape[1], one


class Context:
    """Sketch of A (Alg. 3 initialisation) plus the state of later solves."""

    def __init__(self, A, workspace=0, **opts):
        """workspace = k > 0: the context's device memory is one PyTorch
        tensor sized by aplicur_workspace_bytes for solves with up to k
        right-hand sides; a CUDA uint8 tensor: that memory (reusable by later
        contexts once this one is destroyed; at least workspace_bytes(A, k,
        ...) bytes, else the solve fails with E_NOMEM); 0: the library
        allocates it."""
        self.lib = L.load()
        self.mat, self._keep = _mat(A)
        self.m, self.n = int(self.mat.m), int(self.mat.n)
        self.opts = make_opts(**opts)
        self.workspace = None
        ws, ws_bytes = None, 0
        if isinstance(workspace, torch.Tensor):
            if not workspace.is_cuda or workspace.dtype != torch.uint8 or not workspace.is_contiguous():
                raise ValueError("workspace tensor must be a contiguous CUDA uint8 tensor")
            self.workspace = workspace
            ws, ws_bytes = workspace.data_ptr(), workspace.numel()
        elif workspace:
            ws_bytes = self.lib.aplicur_workspace_bytes(C.byref(self.mat), int(workspace), C.byref(self.opts),
                                                        _stream())
            L.check(int(ws_bytes) if ws_bytes < 0 else 0)
            self.workspace = torch.empty(int(ws_bytes), dtype=torch.uint8, device=_device(A))
            ws = self.workspace.data_ptr()
        ptr = C.c_void_p()
        L.check(self.lib.aplicur_sketch(C.byref(self.mat), C.byref(self.opts), ws, int(ws_bytes), _stream(),
                                        C.byref(ptr)))
        self.ptr = ptr

    def solve(self, B, X0=None):
        Bt, k, one = _cols(B, self.m, "B")
        if X0 is not None:
            Xt, _, _ = _cols(X0, self.n, "X0")
            Xt = Xt.clone()
        else:
            Xt = torch.empty((k, self.n), dtype=torch.float64, device=Bt.device)
        info = L.Info()
        code = L.check(self.lib.aplicur_solve(self.ptr, Bt.data_ptr(), self.m, k, Xt.data_ptr(), self.n,
                                              int(X0 is not None), C.byref(info), _stream()))
        X = Xt.t()
        return (X.reshape(-1) if one else X), info

    def solve_backward(self, X, B, G, want_dA=True):
        """Z = (A^T A + mu I)^{-1} G, dB = A Z, dA = (B - A X) Z^T - (A Z) X^T."""
        Xt, k, one = _cols(X, self.n, "X")
        Bt, _, _ = _cols(B, self.m, "B")
        Gt, _, _ = _cols(G, self.n, "G")
        dev = Xt.device
        Zt = torch.empty((k, self.n), dtype=torch.float64, device=dev)
        dBt = torch.empty((k, self.m), dtype=torch.float64, device=dev)
        dA = None
        dA_ptr, ldda = None, 0
        if want_dA:
            if self.mat.format == L.CSR:
                dA = torch.empty(int(self.mat.nnz), dtype=torch.float64, device=dev)
            elif self.mat.format == L.DENSE_COL:  # dA in A's (column-major) layout
                dAt = torch.empty((self.n, self.m), dtype=torch.float64, device=dev)
                dA, ldda = dAt.t(), self.m
            else:
                dA = torch.empty((self.m, self.n), dtype=torch.float64, device=dev)
                ldda = self.n
            dA_ptr = dA.data_ptr()
        info = L.Info()
        L.check(self.lib.aplicur_solve_backward(self.ptr, Xt.data_ptr(), self.n, Bt.data_ptr(), self.m,
                                                Gt.data_ptr(), self.n, k, Zt.data_ptr(), self.n, dBt.data_ptr(),
                                                self.m, dA_ptr, ldda, C.byref(info), _stream()))
        Z, dB = Zt.t(), dBt.t()
        if one:
            Z, dB = Z.reshape(-1), dB.reshape(-1)
        return Z, dB, dA, info

    def matvec(self, x, trans=False):
        rows_in, rows_out = (self.m, self.n) if trans else (self.n, self.m)
        x = x.to(torch.float64).contiguous()
        if x.numel() != rows_in:
            raise ValueError("x has the wrong length")
        y = torch.empty(rows_out, dtype=torch.float64, device=x.device)
        L.check(self.lib.aplicur_matvec(self.ptr, int(bool(trans)), x.data_ptr(), y.data_ptr(), _stream()))
        return y

    def matmat(self, X, trans=False, prec=0):
        """A X (or A^T X) for the columns of X (rows x k, or a vector); prec
        1 / 2: the FP32 / BF16 products of the low-precision phases."""
        rows_in, rows_out = (self.m, self.n) if trans else (self.n, self.m)
        Xt, k, one = _cols(X, rows_in, "X")
        Yt = torch.empty((k, rows_out), dtype=torch.float64, device=Xt.device)
        L.check(self.lib.aplicur_matmat(self.ptr, int(bool(trans)), Xt.data_ptr(), rows_in, k, Yt.data_ptr(),
                                        rows_out, int(prec), _stream()))
        Y = Yt.t()
        return Y.reshape(-1) if one else Y

    def time_matmat(self, X, trans=False, prec=0, reps=20, flush=None):
        """Mean duration (us) of the blocked product kernel for the columns
        of X (rows x k, k <= 64); flush as in time_product."""
        rows_in, rows_out = (self.m, self.n) if trans else (self.n, self.m)
        Xt, k, _ = _cols(X, rows_in, "X")
        Yt = torch.empty((k, rows_out), dtype=torch.float64, device=Xt.device)
        us = C.c_double()
        fptr, fbytes = (flush.data_ptr(), flush.numel() * flush.element_size()) if flush is not None else (None, 0)
        L.check(self.lib.aplicur_time_matmat(self.ptr, int(bool(trans)), Xt.data_ptr(), rows_in, k, Yt.data_ptr(),
                                             rows_out, int(prec), int(reps), fptr, int(fbytes), _stream(),
                                             C.byref(us)))
        return us.value

    def precond_apply(self, z, trans=False):
        """P^{-1} z (trans: P^{-T} z) with the last preconditioner built."""
        z = z.to(torch.float64).contiguous()
        if z.numel() != self.n:
            raise ValueError("z must have n entries")
        y = torch.empty(self.n, dtype=torch.float64, device=z.device)
        L.check(self.lib.aplicur_precond_apply(self.ptr, int(bool(trans)), z.data_ptr(), y.data_ptr(), _stream()))
        return y

    def time_product(self, x, trans=False, reps=100, flush=None):
        """Mean duration (us) of one launch of the A (or A^T) product kernel,
        A and A^T products alternating; x has n entries.  flush: a device
        buffer (overwritten) read and written before each round, for
        cold-cache timing."""
        x = x.to(torch.float64).contiguous()
        if x.numel() != self.n:
            raise ValueError("x must have n entries")
        y = torch.empty(self.m, dtype=torch.float64, device=x.device)
        us = C.c_double()
        fptr, fbytes = (flush.data_ptr(), flush.numel() * flush.element_size()) if flush is not None else (None, 0)
        L.check(self.lib.aplicur_time_product(self.ptr, int(bool(trans)), x.data_ptr(), y.data_ptr(), int(reps),
                                              fptr, int(fbytes), _stream(), C.byref(us)))
        return us.value

    def query(self, what):
        """Read internal state (see aplicur_ctx_query in include/aplicur.h)."""
        kinds = {1: np.float64, 2: np.int32, 3: np.int32, 4: np.float64, 5: np.int32, 6: np.int32,
                 7: np.float64, 8: np.int32, 9: np.int32, 10: np.int64, 11: np.float64, 12: np.int32,
                 13: np.float64, 14: np.int32, 15: np.float64}
        nbytes = self.lib.aplicur_ctx_query(self.ptr, what, None, 0)
        L.check(int(nbytes) if nbytes < 0 else 0)
        buf = (C.c_char * max(int(nbytes), 1))()
        self.lib.aplicur_ctx_query(self.ptr, what, buf, int(nbytes))
        return np.frombuffer(bytes(buf)[:int(nbytes)], dtype=kinds[what]).copy()

    def sizes(self):
        m, n, s, xi, rank, outer, r = self.query(10).tolist()
        return dict(m=m, n=n, s=s, xi=xi, rank=rank, outer=outer, r=r)

    def close(self):
        if getattr(self, "ptr", None):
            self.lib.aplicur_ctx_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def sketch_noalloc(A, Y=None, **opts):
    """Y = S A (s x n, FP64) through aplicur_sketch_noalloc: no context and no
    device allocation inside the library (Y is allocated here unless given)."""
    lib = L.load()
    mat, keep = _mat(A)
    o = make_opts(**opts)
    s = max(1, min(int(mat.m), math.ceil(1.1 * o.block - 1e-12)))
    if Y is None:
        Y = torch.empty((s, int(mat.n)), dtype=torch.float64, device=_device(A))
    if Y.shape != (s, int(mat.n)) or not Y.is_contiguous() or Y.dtype != torch.float64:
        raise ValueError(f"Y must be a contiguous FP64 ({s}, {int(mat.n)}) tensor")
    L.check(lib.aplicur_sketch_noalloc(C.byref(mat), C.byref(o), Y.data_ptr(), _stream()))
    return Y


PROF_KINDS = ("AX_f64", "ATX_f64", "AX_f32", "ATX_f32", "AX_bf16", "ATX_bf16")


def prof_products(enable=True):
    """Switch event timing of the blocked product kernel inside solves on or
    off (aplicur_prof_products)."""
    L.check(L.load().aplicur_prof_products(int(bool(enable))))


def prof_read():
    """Read and clear the product-kernel event record: {kind: (launches,
    mean microseconds, untimed launches)} for the kinds with any launch."""
    lib = L.load()
    n = len(PROF_KINDS)
    cnt, tot, unt = (C.c_int64 * n)(), (C.c_double * n)(), (C.c_int64 * n)()
    L.check(lib.aplicur_prof_read(cnt, tot, unt))
    return {k: (int(cnt[i]), tot[i] / cnt[i] if cnt[i] else float("nan"), int(unt[i]))
            for i, k in enumerate(PROF_KINDS) if cnt[i] or unt[i]}


def sketch(A, **opts):
    return Context(A, **opts)


def workspace_bytes(A, nrhs, **opts):
    """Bytes of device memory a context of A needs for solves with up to nrhs
    right-hand sides (aplicur_workspace_bytes: one measuring set-up run)."""
    lib = L.load()
    mat, keep = _mat(A)
    o = make_opts(**opts)
    n = lib.aplicur_workspace_bytes(C.byref(mat), int(nrhs), C.byref(o), _stream())
    L.check(int(n) if n < 0 else 0)
    del keep
    return int(n)


def lstsq(A, B, **opts):
    """min ||A X - B||^2 + mu ||X||^2 by APLICUR (precond=False: plain LSQR)."""
    with Context(A, **opts) as ctx:
        return ctx.solve(B)


class LstsqFunction(torch.autograd.Function):
    """X = argmin ||A X - B||^2 + mu ||X||^2 with gradients for A and B
    through the adjoint solve of the library (aplicur_solve_backward).

    apply(a_val, B, structure, opts): a_val is the dense A (CUDA tensor) or the
    values of a CSR matrix whose row_ptr/col_idx/shape come from `structure`
    (a CSRMatrix, None for dense A); the gradient of a_val is dense (m x n) or
    lives on the sparsity pattern (nnz values)."""

    @staticmethod
    def forward(fctx, a_val, B, structure, opts):
        A = a_val if structure is None else CSRMatrix(structure.row_ptr, structure.col_idx, a_val, structure.shape)
        ctx = Context(A, **opts)
        X, info = ctx.solve(B)
        L.check(info.status)
        fctx.lib_ctx = ctx
        fctx.a_dtype, fctx.b_dtype = a_val.dtype, B.dtype
        fctx.save_for_backward(X, B)
        return X

    @staticmethod
    def backward(fctx, G):
        X, B = fctx.saved_tensors
        want_dA = bool(fctx.needs_input_grad[0])
        _, dB, dA, _ = fctx.lib_ctx.solve_backward(X, B, G.contiguous(), want_dA=want_dA)
        gA = dA.to(fctx.a_dtype) if want_dA else None
        gB = dB.to(fctx.b_dtype).reshape(B.shape) if fctx.needs_input_grad[1] else None
        return gA, gB, None, None


def lstsq_autograd(A, B, **opts):
    """Differentiable lstsq: A is a dense CUDA tensor or a CSRMatrix (its
    `val` may require grad), B a CUDA tensor (m,) or (m, k)."""
    if isinstance(A, CSRMatrix):
        return LstsqFunction.apply(A.val, B, A, opts)
    return LstsqFunction.apply(A, B, None, opts)


def batched_workspace_bytes(As, nrhs, workers=0, tune=True, graphs=True, **opts):
    """Bytes of the workspace solve_batched(..., workspace=...) needs."""
    lib = L.load()
    o = make_opts(workers=workers, tune=tune, graphs=graphs, **opts)
    mats, keep = [], []
    for A in As:
        st, kp = _mat(A)
        mats.append(st)
        keep.append(kp)
    marr = (L.Mat * len(As))(*mats)
    n = lib.aplicur_batched_workspace_bytes(len(As), marr, int(nrhs), C.byref(o), _stream())
    if n < 0:
        L.check(int(n))
    return int(n)


def solve_batched(As, Bs, workers=0, tune=True, graphs=True, workspace=None, **opts):
    """Independent problems min ||A_p X_p - B_p||^2 + mu ||X_p||^2 (same
    options, same number of right-hand sides), solved concurrently by the
    library's worker streams; returns ([X_p], [info_p]).  workspace: an
    optional device tensor (uint8, 256-byte aligned) of at least
    batched_workspace_bytes bytes that every context is carved from."""
    lib = L.load()
    o = make_opts(workers=workers, tune=tune, graphs=graphs, **opts)
    mats, keep = [], []
    for A in As:
        st, kp = _mat(A)
        mats.append(st)
        keep.append(kp)
    p = len(As)
    MatArr = L.Mat * p
    marr = MatArr(*mats)
    cols = [_cols(B, int(A.shape[0]), "B") for A, B in zip(As, Bs)]
    k = cols[0][1]
    if any(c[1] != k for c in cols):
        raise ValueError("every problem needs the same number of right-hand sides")
    Xs = [torch.empty((k, int(A.shape[1])), dtype=torch.float64, device=cols[0][0].device) for A in As]
    bptr = (C.c_void_p * p)(*[c[0].data_ptr() for c in cols])
    xptr = (C.c_void_p * p)(*[x.data_ptr() for x in Xs])
    ldb = (C.c_int64 * p)(*[int(A.shape[0]) for A in As])
    ldx = (C.c_int64 * p)(*[int(A.shape[1]) for A in As])
    infos = (L.Info * p)()
    ws_ptr, ws_bytes = (workspace.data_ptr(), workspace.numel() * workspace.element_size()) if workspace is not None \
        else (None, 0)
    L.check(lib.aplicur_solve_batched(p, marr, bptr, ldb, k, xptr, ldx, C.byref(o), ws_ptr, ws_bytes, infos,
                                      _stream()))
    outs = [x.t() for x in Xs]
    if cols[0][2]:
        outs = [x.reshape(-1) for x in outs]
    return outs, list(infos)
