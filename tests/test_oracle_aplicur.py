"""Pins of the oracle's full procedure (Alg. 3): the solution is the unique
minimiser (dense QR), the normal-equation invariant holds, the multi-RHS
reading is column-by-column, and degenerate inputs behave."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.aplicur import Options, Trace, aplicur, ne_residual
from oracle.dense import adjoint, gram_solve, solve_dense_qr, solve_normal
from workloads import synth


def _floor(A, mu):
    Ad = A.toarray() if sp.issparse(A) else A
    s = np.linalg.svd(Ad, compute_uv=False)
    kappa = math.sqrt((s[0] ** 2 + mu) / (s[-1] ** 2 + mu))
    return kappa


def test_workload1_small():
    w = synth.workload(1, 0.25)
    tr = Trace()
    x = aplicur(w.A, w.B, w.mu, Options(block=w.block, tol_ne=w.tol), tr)
    eta = ne_residual(w.A, w.B, x, w.mu)
    assert eta <= w.tol
    xr = solve_dense_qr(w.A, w.B, w.mu)
    # the normal-equation residual pins x only up to eta ||A^T b|| / sigma_min^2
    smin = np.linalg.svd(w.A, compute_uv=False)[-1]
    bound = eta * np.linalg.norm(w.A.T @ w.B) / smin ** 2
    assert np.linalg.norm(x - xr) <= 2 * bound + 1e-9 * np.linalg.norm(xr)
    assert tr.ranks == sorted(tr.ranks) and tr.rebuild[0] and tr.rebuild[-1]
    # at a tight tolerance the iterate reaches the dense-QR solution
    kappa = _floor(w.A, w.mu)
    x2 = aplicur(w.A, w.B, w.mu, Options(block=w.block, tol_ne=1e-14))
    assert np.linalg.norm(x2 - xr) / np.linalg.norm(xr) <= 1e3 * kappa * 2.2e-16


def test_workload2_small_sparse():
    w = synth.workload(2, 0.02)
    tr = Trace()
    x = aplicur(w.A, w.B, w.mu, Options(block=w.block, tol_ne=w.tol), tr)
    assert ne_residual(w.A, w.B, x, w.mu) <= w.tol
    xr = solve_normal(w.A.toarray(), w.B, w.mu)
    assert np.linalg.norm(x - xr) / np.linalg.norm(xr) <= 1e-6
    A = w.A
    np.testing.assert_allclose(A.T @ (w.B - A @ x), w.mu * x,
                               atol=1e-7 * np.linalg.norm(A.T @ w.B))


def test_residual_monotone_across_phases():
    r = np.random.default_rng(0)
    sigma = np.concatenate([np.logspace(2, -2, 10), np.logspace(-4.8, -5, 40)])
    A = synth.dense_svd(r, 200, 50, sigma)
    xs, b = synth.consistent_x(r, A, noise=1e-2)
    mu = 1e-4
    opts = Options(block=5, tol_ne=1e-12)
    # true augmented residual after each phase must not increase (Sec. 3.2)
    res = []
    orig = aplicur.__globals__["plsqr_phase"]

    def spy(A_, delta, b_, x, pinv, **kw):
        out = orig(A_, delta, b_, x, pinv, **kw)
        xn = out[0]
        res.append(math.hypot(np.linalg.norm(b_ - A_ @ xn), delta * np.linalg.norm(xn)))
        return out
    aplicur.__globals__["plsqr_phase"] = spy
    try:
        x = aplicur(A, b, mu, opts)
    finally:
        aplicur.__globals__["plsqr_phase"] = orig
    assert len(res) >= 2
    assert all(res[i + 1] <= res[i] * (1 + 1e-12) for i in range(len(res) - 1))
    np.testing.assert_allclose(x, solve_dense_qr(A, b, mu), rtol=1e-6)


def test_multi_rhs_is_columnwise():
    w = synth.workload(1, 0.2)
    B = np.column_stack([w.B, np.random.default_rng(1).standard_normal(w.B.shape[0])])
    X = aplicur(w.A, B, 1e-6, Options(block=4, tol_ne=1e-9))
    for k in range(2):
        xk = aplicur(w.A, B[:, k], 1e-6, Options(block=4, tol_ne=1e-9))
        np.testing.assert_array_equal(X[:, k], xk)


def test_zero_rhs():
    A = np.random.default_rng(2).standard_normal((30, 8))
    x = aplicur(A, np.zeros(30), 0.1, Options(block=2))
    assert np.all(x == 0)


def test_rank_cap_same_solution():
    w = synth.workload(2, 0.02)
    xr = solve_normal(w.A.toarray(), w.B, w.mu)
    x = aplicur(w.A, w.B, w.mu, Options(block=w.block, tol_ne=1e-9, max_rank=3 * w.block))
    assert ne_residual(w.A, w.B, x, w.mu) <= 1e-9
    assert np.linalg.norm(x - xr) / np.linalg.norm(xr) <= 1e-6


def test_rank_cap_limits_the_last_increment():
    """A cap that is not a multiple of the block ends the growth exactly at
    the cap (the last increment is cut), like the GPU library's rank cap."""
    A = synth.dense_svd(np.random.default_rng(9), 300, 80, 10.0 ** (-8 * np.arange(80) / 79))
    b = np.random.default_rng(10).standard_normal(300)
    tr = Trace()
    aplicur(A, b, 1e-12, Options(block=10, tol_ne=1e-10, max_rank=25), tr)
    assert tr.ranks == [10, 20, 25]
    assert tr.rebuild[-1]


def test_adjoint_matches_finite_differences():
    r = np.random.default_rng(3)
    m, n, k, mu = 30, 8, 2, 0.05
    A = r.standard_normal((m, n))
    B = r.standard_normal((m, k))

    def loss(A_, B_):
        X = solve_dense_qr(A_, B_, mu)
        return float(np.sum(X * X))
    X = solve_dense_qr(A, B, mu)
    Z, dB, dA = adjoint(A, X, B, 2.0 * X, mu)
    # normal-equations route for Z
    np.testing.assert_allclose(Z, gram_solve(A, 2.0 * X, mu), rtol=1e-10)
    h = 1e-3
    for _ in range(6):
        D = r.standard_normal((m, n)); D /= np.linalg.norm(D)
        fd = (loss(A + h * D, B) - loss(A - h * D, B)) / (2 * h)
        assert abs(fd - np.sum(dA * D)) <= 1e-5 * max(1.0, abs(fd))
        E = r.standard_normal((m, k)); E /= np.linalg.norm(E)
        fd = (loss(A, B + h * E) - loss(A, B - h * E)) / (2 * h)
        assert abs(fd - np.sum(dB * E)) <= 1e-5 * max(1.0, abs(fd))


def test_aplicur_gaussian_sketch_reaches_dense_qr():
    """The Gaussian sketch changes the CUR indices, not the solution."""
    r = np.random.default_rng(31)
    A = synth.dense_svd(r, 400, 50, 10.0 ** (-4 * np.arange(50) / 49))
    b = r.standard_normal(400)
    x = aplicur(A, b, 1e-6, Options(block=6, tol_ne=1e-10, sketch="gaussian"))
    xr = solve_dense_qr(A, b, 1e-6)
    assert np.linalg.norm(x - xr) <= 1e-7 * np.linalg.norm(xr)


@pytest.mark.parametrize("schedule", [1, 2])
def test_single_shot_schedules(schedule):
    """Sec. 7.1 variants: one preconditioner build, at the final rank (the rank
    where rho <= eps_cur for the rank-adaptive single shot, the cap for the
    fixed-rank one), followed by the final phase; same solution."""
    r = np.random.default_rng(32)
    A = synth.dense_svd(r, 500, 60, 10.0 ** (-6 * np.arange(60) / 59))
    b = r.standard_normal(500)
    mu, cap = 1e-8, 30
    tr = Trace()
    x = aplicur(A, b, mu, Options(block=5, tol_ne=1e-10, max_rank=cap, schedule=schedule), tr)
    assert tr.rebuild == [False] * (len(tr.rebuild) - 1) + [True]
    assert len(tr.phase_iters) >= 1
    if schedule == 2:
        assert tr.ranks[-1] == cap
    else:
        from oracle.aplicur import default_eps_cur
        assert tr.rhos[-1] <= default_eps_cur(mu) or tr.ranks[-1] == cap
        assert all(rho > default_eps_cur(mu) for rho in tr.rhos[:-1])
    xr = solve_dense_qr(A, b, mu)
    assert np.linalg.norm(x - xr) <= 1e-6 * np.linalg.norm(xr)


def test_dependent_columns_end_rank_growth():
    """Root-exponential decay to 1e-13 with mu = 0: the cross approximation
    reaches columns numerically dependent on C (C^T C not positive definite in
    floating point); by default that step is undone and the growth ends there
    (the rank repeats in the trace), and the solve still reaches its
    tolerance."""
    r = np.random.default_rng(0)
    A = synth.dense_svd(r, 1200, 1000, synth.paper_sigma(1000, "smooth"))
    b = A @ r.standard_normal(1000)
    tr = Trace()
    x = aplicur(A, b, 0.0, Options(block=20, tol_ne=1e-8, max_iter=20000), tr)
    assert tr.ranks[-1] == tr.ranks[-2] and tr.rebuild[-1]
    assert ne_residual(A, b, x, 0.0) <= 1e-8


def test_sketched_cholqr_continues_the_rank_growth():
    """The same set at mu = 1e-10, single-shot schedule 2 (the CUR grows to the
    rank cap of 400 before the one build): by default the breakdown of
    chol(C^T C) at rank 280 ends the growth at 260; with tc = "sketched" T_C
    comes from sketched Cholesky QR (T^T T = C^T C to rounding while the
    plain Cholesky of the final C^T C fails), the ranks reach the cap, and the
    larger P needs fewer iterations to the same tolerance."""
    from oracle.cur import t_c_factor
    r = np.random.default_rng(0)
    A = synth.dense_svd(r, 1200, 1000, synth.paper_sigma(1000, "smooth"))
    b = A @ r.standard_normal(1000)
    mu, opts = 1e-10, dict(block=20, tol_ne=1e-8, max_iter=20000, schedule=2, max_rank=400)
    tr0, tr = Trace(), Trace()
    x0 = aplicur(A, b, mu, Options(**opts), tr0)
    x = aplicur(A, b, mu, Options(tc="sketched", **opts), tr)
    assert tr0.ranks[-1] == tr0.ranks[-2] == 260
    assert tr.ranks == list(range(20, 401, 20))
    C = A[:, tr.J]
    with pytest.raises(np.linalg.LinAlgError):
        np.linalg.cholesky(C.T @ C)
    T = t_c_factor(C, Options().seed)
    assert T is not None and np.linalg.norm(C.T @ C - T.T @ T) <= 1e-14 * np.linalg.norm(C) ** 2
    assert ne_residual(A, b, x0, mu) <= 1e-8 and ne_residual(A, b, x, mu) <= 1e-8
    assert tr.iters < tr0.iters
