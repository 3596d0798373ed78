"""Pins of the oracle's SVD-free preconditioner (Alg. 8, Sec. 3.1, mu = 0).

What fixes it independently of its own formulas:
* Lemma 5.2: A P~^{-1} and A P^{-1} (SVD-based, same target level) have the
  same singular values, although P~ != P;
* the direct form P~ = s^{-1} Q_R M Q_R^T + (I - Q_R Q_R^T) with
  M = T_C A(I,J)^{-1} T_R^T is the inverse of the applied operator;
* the transpose apply is the adjoint of the forward apply;
* the Corollary after Lemma 5.2: one LSQR phase with P~ and one with P from the
  same start have the same residual estimates phibar_k at every k (and with
  P~^{-1} wrongly used for both applies they do not);
* the full solve reaches the dense-QR minimiser.
"""
import numpy as np
import pytest

from oracle import rng
from oracle.aplicur import Options, Trace, aplicur, ne_residual, sketch_rows
from oracle.cur import (Preconditioner, SvdFreePreconditioner, augment_cur, augment_qr,
                        core_and_residual, rho_estimate)
from oracle.dense import solve_dense_qr
from oracle.lsqr import plsqr_phase
from workloads import synth


def _problem(m=300, n=120, decades=6.0, seed=3):
    r = np.random.default_rng(seed)
    A = synth.dense_svd(r, m, n, 10.0 ** (-decades * np.arange(n) / (n - 1)))
    b = A @ r.standard_normal(n) + 1e-6 * r.standard_normal(m)
    return A, b


def _cur(A, ell, block=20, seed=7):
    """CUR factors at rank ell by the oracle's own Alg. 7 / Alg. 9 steps."""
    m, n = A.shape
    Y = rng.sparse_sign_matrix(seed, sketch_rows(block, m), m) @ A
    probes = rng.gaussian_probes(seed, n, 10)
    I = J = np.zeros(0, np.int64)
    C = W = R = Q = T = None
    E_row = Y.copy()
    while len(J) < ell:
        Ip, Jp, done = augment_cur(A, E_row, I, J, C, W, R, min(block, ell - len(J)))
        I, J = np.concatenate([I, Ip]), np.concatenate([J, Jp])
        C, W, R, E_row = core_and_residual(A, Y, I, J)
        Q, T = augment_qr(Q, T, A[Ip, :].T)
        if done:
            break
    return C, W, Q, T, rho_estimate(E_row, probes)


def _svd_inverse(C, W, Q, T, target):
    """P^{-1} of Alg. 2 at mu = 0 with its target level replaced by ``target``."""
    P = Preconditioner(C, W, Q, T, 0.0)
    return np.eye(Q.shape[0]) + (P.V * (target / P.Lam - 1.0)) @ P.V.T, P


def test_lemma_equal_singular_values():
    A, _ = _problem()
    C, W, Q, T, rho = _cur(A, 40)
    Pf = SvdFreePreconditioner(C, W, Q, T, rho, 3e-7)
    assert Pf.target == rho
    Pi, _ = _svd_inverse(C, W, Q, T, Pf.target)
    Pfi = Pf.dense_inverse()
    # the two operators differ (by a right orthogonal factor) ...
    assert np.linalg.norm(Pfi - Pi) > 1e-3 * np.linalg.norm(Pi)
    # ... which is orthogonal: Pi^{-1} Pfi has unit singular values
    Wo = np.linalg.solve(Pi, Pfi)
    assert np.allclose(np.linalg.svd(Wo, compute_uv=False), 1.0, atol=1e-8)
    s1 = np.linalg.svd(A @ Pfi, compute_uv=False)
    s2 = np.linalg.svd(A @ Pi, compute_uv=False)
    assert np.max(np.abs(s1 - s2)) <= 1e-9 * s2[0]


def test_direct_form_is_the_inverse():
    A, _ = _problem(seed=5)
    C, W, Q, T, rho = _cur(A, 40)
    Pf = SvdFreePreconditioner(C, W, Q, T, rho, 3e-7)
    n = A.shape[1]
    T_C = np.linalg.cholesky(C.T @ C).T
    M = T_C @ np.linalg.inv(W) @ T.T
    Pdirect = (Q @ M @ Q.T) / rho + np.eye(n) - Q @ Q.T
    E = Pdirect @ Pf.dense_inverse() - np.eye(n)
    assert np.linalg.norm(E) <= 1e-8


def test_transpose_apply_is_the_adjoint():
    A, _ = _problem(seed=6)
    C, W, Q, T, rho = _cur(A, 40)
    Pf = SvdFreePreconditioner(C, W, Q, T, rho, 3e-7)
    n = A.shape[1]
    F = np.column_stack([Pf.inv(e) for e in np.eye(n)])
    G = np.column_stack([Pf.inv_t(e) for e in np.eye(n)])
    assert np.linalg.norm(G - F.T) <= 1e-12 * np.linalg.norm(F)
    assert np.linalg.norm(F - F.T) > 1e-3 * np.linalg.norm(F)  # not symmetric


def test_corollary_equal_residual_histories():
    A, b = _problem(seed=8)
    C, W, Q, T, rho = _cur(A, 40)
    Pf = SvdFreePreconditioner(C, W, Q, T, rho, 3e-7)
    Pi, _ = _svd_inverse(C, W, Q, T, Pf.target)
    x0 = np.zeros(A.shape[1])
    # 12 steps: without re-orthogonalisation the two finite-precision
    # recurrences part by rounding later (1e-13 up to step 14, 1e-6 after)
    kw = dict(eps_lsqr=0.0, tol_ne=0.0, max_iter=12)
    h_free, h_svd, h_wrong = [], [], []
    plsqr_phase(A, 0.0, b, x0, Pf.inv, pinv_t=Pf.inv_t, history=h_free, **kw)
    plsqr_phase(A, 0.0, b, x0, lambda z: Pi @ z, history=h_svd, **kw)
    plsqr_phase(A, 0.0, b, x0, Pf.inv, history=h_wrong, **kw)
    h_free, h_svd, h_wrong = map(np.array, (h_free, h_svd, h_wrong))
    assert len(h_free) == len(h_svd) == 12
    assert np.max(np.abs(h_free - h_svd) / h_svd) <= 1e-10
    # applying P~^{-1} in place of P~^{-T} is another (wrong) recurrence
    assert np.max(np.abs(h_wrong[:len(h_svd)] - h_svd[:len(h_wrong)]) / h_svd[:len(h_wrong)]) > 1.0


def test_svdfree_solve_reaches_the_minimiser():
    w = synth.workload(1, 0.25)
    tr = Trace()
    x = aplicur(w.A, w.B, 0.0, Options(block=w.block, tol_ne=w.tol, precond="svdfree"), tr)
    eta = ne_residual(w.A, w.B, x, 0.0)
    assert eta <= w.tol
    xr = solve_dense_qr(w.A, w.B, 0.0)
    smin = np.linalg.svd(w.A, compute_uv=False)[-1]
    bound = eta * np.linalg.norm(w.A.T @ w.B) / smin ** 2
    assert np.linalg.norm(x - xr) <= 2 * bound + 1e-9 * np.linalg.norm(xr)
    # the target level is rho at each rebuild (Alg. 8), not below eps_cur
    built = [max(r, 3e-7) for r, f in zip(tr.rhos, tr.rebuild) if f]
    assert tr.sigma_hat == built
    # the same CUR sequence as the SVD-based run (P does not enter it)
    tr2 = Trace()
    aplicur(w.A, w.B, 0.0, Options(block=w.block, tol_ne=w.tol), tr2)
    assert tr.ranks == tr2.ranks and np.array_equal(tr.J, tr2.J)


def test_target_floor():
    A, _ = _problem(seed=9)
    C, W, Q, T, rho = _cur(A, 20)
    assert SvdFreePreconditioner(C, W, Q, T, 0.0, 3e-7).target == 3e-7
    assert SvdFreePreconditioner(C, W, Q, T, 1e-12, 3e-7).target == 3e-7


def test_full_rank_sparse_solve():
    """Rank up to n (rho at rounding level): the floor keeps the target at
    eps_cur and the solve reaches the minimiser (sparse A, mu = 0)."""
    A = synth.sparse_scaled(np.random.default_rng(3), 4000, 400, 10, 4.0)
    b = np.random.default_rng(5).standard_normal(4000)
    tr = Trace()
    x = aplicur(A, b, 0.0, Options(block=20, tol_ne=1e-8, precond="svdfree"), tr)
    assert tr.ranks[-1] == 400 and tr.rhos[-1] < 3e-7 and tr.sigma_hat[-1] == 3e-7
    Ad = A.toarray()
    assert ne_residual(Ad, b, x, 0.0) <= 1e-8
    xr = solve_dense_qr(Ad, b, 0.0)
    assert np.linalg.norm(x - xr) <= 1e-6 * np.linalg.norm(xr)


def test_svdfree_needs_mu_zero():
    A, b = _problem(m=60, n=20)
    with pytest.raises(ValueError):
        aplicur(A, b, 1e-4, Options(precond="svdfree"))
