"""Pins of the oracle's LSQR phase (Sec. 2.2): residual estimate, monotonicity,
finite termination, equivalence with CG on the normal equations, and the
solution against dense QR of the augmented problem (Sec. 2.1)."""
import math

import numpy as np
import pytest

from oracle.aplicur import lsqr_plain, ne_residual
from oracle.dense import solve_dense_qr, solve_normal
from oracle.lsqr import plsqr_phase


def _problem(m, n, cond, seed):
    r = np.random.default_rng(seed)
    U, _ = np.linalg.qr(r.standard_normal((m, n)))
    V, _ = np.linalg.qr(r.standard_normal((n, n)))
    s = np.logspace(0, -math.log10(cond), n)
    return (U * s) @ V.T, r.standard_normal(m)


@pytest.mark.parametrize("mu", [0.0, 1e-2])
def test_plain_lsqr_matches_qr(mu):
    A, b = _problem(80, 20, 1e3, 1)
    x, it = lsqr_plain(A, b, mu, tol_ne=1e-13)
    xr = solve_dense_qr(A, b, mu)
    np.testing.assert_allclose(x, xr, rtol=1e-8, atol=1e-8 * np.linalg.norm(xr))
    # normal-equation invariant A^T (b - A x) = mu x
    np.testing.assert_allclose(A.T @ (b - A @ x), mu * x, atol=1e-11 * np.linalg.norm(A.T @ b))
    assert ne_residual(A, b, x, mu) <= 1e-13


def test_dense_routes_agree():
    A, b = _problem(60, 15, 10.0, 2)
    np.testing.assert_allclose(solve_dense_qr(A, b, 0.3), solve_normal(A, b, 0.3), rtol=1e-12)


def test_phibar_is_true_residual_and_monotone():
    A, b = _problem(70, 25, 1e2, 3)
    delta = 0.1
    hist = []
    plsqr_phase(A, delta, b, np.zeros(25), None, eps_lsqr=0, tol_ne=0, max_iter=12, history=hist)
    assert all(hist[i + 1] <= hist[i] * (1 + 1e-14) for i in range(len(hist) - 1))
    for j in (1, 4, 9):
        xj, it, _ = plsqr_phase(A, delta, b, np.zeros(25), None, eps_lsqr=0, tol_ne=0, max_iter=j)
        true = math.sqrt(np.linalg.norm(b - A @ xj) ** 2 + (delta * np.linalg.norm(xj)) ** 2)
        assert abs(true - hist[j - 1]) <= 1e-10 * np.linalg.norm(b)


def test_finite_termination_distinct_singular_values():
    # A with 3 distinct singular values: LSQR (= CG on A^T A) ends in 3 steps
    r = np.random.default_rng(4)
    U, _ = np.linalg.qr(r.standard_normal((40, 12)))
    V, _ = np.linalg.qr(r.standard_normal((12, 12)))
    s = np.repeat([3.0, 1.0, 0.2], 4)
    A = (U * s) @ V.T
    b = r.standard_normal(40)
    x3, _, _ = plsqr_phase(A, 0.0, b, np.zeros(12), None, eps_lsqr=0, tol_ne=0, max_iter=3)
    np.testing.assert_allclose(x3, solve_dense_qr(A, b, 0.0), rtol=1e-9)


def test_equivalent_to_cg_on_normal_equations():
    A, b = _problem(50, 10, 5.0, 5)
    H, g = A.T @ A, A.T @ b
    x = np.zeros(10); r = g.copy(); p = r.copy()
    cg = []
    for _ in range(5):  # textbook conjugate gradients on A^T A x = A^T b
        Hp = H @ p
        a = (r @ r) / (p @ Hp)
        x = x + a * p
        rn = r - a * Hp
        p = rn + ((rn @ rn) / (r @ r)) * p
        r = rn
        cg.append(x.copy())
    for k in (1, 3, 5):
        xk, _, _ = plsqr_phase(A, 0.0, b, np.zeros(10), None, eps_lsqr=0, tol_ne=0, max_iter=k)
        np.testing.assert_allclose(xk, cg[k - 1], rtol=1e-9, atol=1e-12)


def test_preconditioning_changes_iterates_not_solution():
    A, b = _problem(60, 16, 1e4, 6)
    mu = 1e-6
    r = np.random.default_rng(7)
    G = r.standard_normal((16, 16))
    Pi = np.eye(16) + 0.5 * (G @ G.T) / 16  # symmetric positive definite P^{-1}
    x_prec, _, _ = plsqr_phase(A, math.sqrt(mu), b, np.zeros(16), lambda z: Pi @ z,
                               eps_lsqr=0, tol_ne=1e-13, atb_norm=np.linalg.norm(A.T @ b),
                               pnorm=np.linalg.norm(np.linalg.inv(Pi), 2), max_iter=500)
    x_ref = solve_dense_qr(A, b, mu)
    np.testing.assert_allclose(x_prec, x_ref, rtol=1e-7, atol=1e-7 * np.linalg.norm(x_ref))
    x_few, _, _ = plsqr_phase(A, math.sqrt(mu), b, np.zeros(16), lambda z: Pi @ z,
                              eps_lsqr=0, tol_ne=0, max_iter=2)
    x_few_plain, _, _ = plsqr_phase(A, math.sqrt(mu), b, np.zeros(16), None,
                                    eps_lsqr=0, tol_ne=0, max_iter=2)
    assert np.linalg.norm(x_few - x_few_plain) > 1e-6


def test_warm_start_restart_keeps_residual_monotone():
    A, b = _problem(60, 20, 1e3, 8)
    delta = 0.05
    x = np.zeros(20)
    prev = np.inf
    for _ in range(6):
        x, _, _ = plsqr_phase(A, delta, b, x, None, eps_lsqr=0, tol_ne=0, max_iter=4)
        res = math.hypot(np.linalg.norm(b - A @ x), delta * np.linalg.norm(x))
        assert res <= prev * (1 + 1e-13)
        prev = res
