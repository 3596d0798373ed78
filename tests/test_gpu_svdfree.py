"""The SVD-free preconditioner (Alg. 8, mu = 0) of the HIP library against the
oracle: the middle matrix H = t M^{-1} - I of the apply element by element,
the target level, the CUR sequence, and whole solves (dense, and CSR up to
full rank) against the dense-QR minimiser."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

from oracle import rng as orng
from oracle.aplicur import Options, Trace, aplicur, ne_residual, sketch_rows
from oracle.cur import (SvdFreePreconditioner, augment_cur, augment_qr, core_and_residual,
                        rho_estimate)
from oracle.dense import solve_dense_qr
from workloads import synth

from bounds import check_solution

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV, dtype=dtype)


def _problem(kind, seed):
    r = np.random.default_rng(seed)
    if kind == "dense":
        A = synth.dense_svd(r, 600, 90, 10.0 ** (-3.0 * np.arange(90) / 89))
    else:
        A = synth.sparse_scaled(r, 3000, 200, 8, 2.0)
    return A, r.standard_normal(A.shape[0])


def _gpu(lib, A, kind):
    return _t(A) if kind == "dense" else lib.CSRMatrix.from_scipy(A, device=DEV, dtype=torch.float64)


def _oracle_steps(A, steps, block, seed=7):
    """The oracle's CUR factors after ``steps`` increments (Alg. 7 / Alg. 9)."""
    m, n = A.shape
    Ad = A.toarray() if hasattr(A, "toarray") else A
    Y = orng.sparse_sign_matrix(seed, sketch_rows(block, m), m) @ A
    Y = Y.toarray() if sp.issparse(Y) else np.asarray(Y)
    probes = orng.gaussian_probes(seed, n, 10)
    I = J = np.zeros(0, np.int64)
    C = W = R = Q = T = None
    E_row = Y.copy()
    for _ in range(steps):
        Ip, Jp, _ = augment_cur(A, E_row, I, J, C, W, R, block)
        I, J = np.concatenate([I, Ip]), np.concatenate([J, Jp])
        C, W, R, E_row = core_and_residual(A, Y, I, J)
        Q, T = augment_qr(Q, T, Ad[Ip, :].T)
    return I, J, C, W, Q, T, rho_estimate(E_row, probes)


@pytest.mark.parametrize("kind", ["dense", "csr"])
def test_middle_matrix_matches_oracle(lib, kind):
    A, b = _problem(kind, 4)
    block, steps = 12, 2
    with lib.Context(_gpu(lib, A, kind), mu=0.0, block=block, max_outer=steps, tol_ne=1e-30,
                     max_iter=200, precond="svdfree") as ctx:
        x, info = ctx.solve(_t(b))
        I, J, rho = ctx.query(6), ctx.query(5), ctx.query(7)
        l = len(J)
        Xg = ctx.query(15).reshape(l, l)  # row-major
        sigma_hat = info.sigma_hat
    Io, Jo, C, W, Q, T, rho_o = _oracle_steps(A, steps, block)
    np.testing.assert_array_equal(J, Jo)
    np.testing.assert_array_equal(I, Io)
    assert abs(rho[-1] - rho_o) <= 1e-10 * rho_o
    Pf = SvdFreePreconditioner(C, W, Q, T, rho_o, 3e-7)
    assert abs(sigma_hat - Pf.target) <= 1e-10 * Pf.target
    H = Pf.target * Pf.Minv - np.eye(l)
    assert np.linalg.norm(Xg - H) <= 1e-8 * np.linalg.norm(H)


@pytest.mark.parametrize("kind", ["dense", "csr"])
def test_svdfree_solve_matches_oracle(lib, kind):
    if kind == "dense":
        w = synth.workload(1, 0.25)
        A, b, tol, block = w.A, w.B, w.tol, w.block
    else:
        A = synth.sparse_scaled(np.random.default_rng(3), 4000, 400, 10, 4.0)
        b = np.random.default_rng(5).standard_normal(4000)
        tol, block = 1e-8, 20
    tr = Trace()
    xo = aplicur(A, b, 0.0, Options(block=block, tol_ne=tol, precond="svdfree"), tr)
    with lib.Context(_gpu(lib, A, kind), mu=0.0, block=block, tol_ne=tol, precond="svdfree") as ctx:
        x, info = ctx.solve(_t(b))
        ranks, rebuild = ctx.query(8), ctx.query(9)
    x = x.cpu().numpy()
    Ad = A.toarray() if hasattr(A, "toarray") else A
    eta = ne_residual(Ad, b, x, 0.0)
    assert info.status == 0 and eta <= tol
    # the same CUR sequence and rebuilds as far as both ran (the solve ends
    # after the phase whose eta meets the tolerance, which rounding may move
    # by one outer step)
    k = min(len(ranks), len(tr.ranks))
    assert abs(len(ranks) - len(tr.ranks)) <= 1
    assert list(ranks[:k]) == tr.ranks[:k] and [bool(f) for f in rebuild[:k]] == tr.rebuild[:k]
    xr = solve_dense_qr(Ad, b, 0.0)
    smin = np.linalg.svd(Ad, compute_uv=False)[-1]
    bound = eta * np.linalg.norm(Ad.T @ b) / smin ** 2
    assert np.linalg.norm(x - xr) <= 2 * bound + 1e-9 * np.linalg.norm(xr)
    assert ne_residual(Ad, b, xo, 0.0) <= tol


def test_svdfree_fp32_phases_and_columns(lib):
    """FP32 LSQR phases with FP64 refinement, and several right-hand sides (one
    column at a time: the blocked apply has the SVD form only)."""
    w = synth.workload(1, 0.25)
    B = np.column_stack([w.B, np.random.default_rng(1).standard_normal(w.A.shape[0])])
    with lib.Context(_t(w.A), mu=0.0, block=w.block, tol_ne=1e-9, precond="svdfree", precision=1) as ctx:
        X, info = ctx.solve(_t(B))
    X = X.cpu().numpy()
    assert info.status == 0
    for k in range(2):
        assert ne_residual(w.A, B[:, k], X[:, k], 0.0) <= 1e-9
    with lib.Context(_t(w.A), mu=0.0, block=w.block, tol_ne=1e-9, precond="svdfree") as ctx:
        x1, _ = ctx.solve(_t(B[:, 1]))
    xr = solve_dense_qr(w.A, B[:, 1], 0.0)
    check_solution(x1.cpu().numpy(), xr, w.A, B[:, 1], 0.0, "SVD-free, second column")


def test_svdfree_rejects_mu(lib):
    A, b = _problem("dense", 2)
    with pytest.raises(Exception, match="SVD-free"):
        lib.Context(_t(A), mu=1e-4, precond="svdfree")
