"""Pins of the oracle's CUR building blocks: LUPP pivots (Alg. 7 selection),
augmentQR (Alg. 9), CUR-CA exactness (Definition 3.1), the rho bound
(Sec. 5.3.1) and the CUR preconditioner (Alg. 2, Theorem 4.1)."""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import rng
from oracle.cur import (Preconditioner, augment_cur, augment_qr, core_and_residual,
                        lupp_pivots, rho_estimate)


def lapack_pivots(X, k):
    lu, piv = sla.lu_factor(X)
    perm = np.arange(X.shape[0])
    for i, p in enumerate(piv):
        perm[i], perm[p] = perm[p], perm[i]
    return perm[:k]


@pytest.mark.parametrize("shape,k", [((50, 8), 8), ((8, 8), 8), ((300, 20), 12), ((20, 30), 20)])
def test_lupp_matches_lapack(shape, k):
    X = np.random.default_rng(shape[0] + k).standard_normal(shape)
    piv, keff = lupp_pivots(X, k)
    assert keff == min(k, *shape)
    np.testing.assert_array_equal(piv, lapack_pivots(X, keff))


def test_lupp_tiny_by_hand():
    # column 0 max |.| is row 2 (value -5); after eliminating, column 1 of the
    # remaining rows is [2 - 1*(-4/-5)... ] worked by hand below
    X = np.array([[1.0, 2.0], [3.0, 1.0], [-5.0, 4.0]])
    # step 0: pivot row 2; l = [1/-5, 3/-5]; row0 col1: 2 - (-0.2)*4 = 2.8,
    #         row1 col1: 1 - (-0.6)*4 = 3.4 -> step 1 pivot row 1
    piv, keff = lupp_pivots(X, 2)
    assert keff == 2 and piv.tolist() == [2, 1]


def test_lupp_first_max_tie_and_exhaustion():
    X = np.array([[1.0, 0.0], [-1.0, 0.0], [1.0, 0.0]])
    piv, keff = lupp_pivots(X, 2)
    assert piv.tolist() == [0] and keff == 1  # first maximal entry; zero second column
    Z = np.zeros((5, 3))
    piv, keff = lupp_pivots(Z, 3)
    assert keff == 0


def test_augment_qr_properties():
    r = np.random.default_rng(1)
    n = 40
    blocks = [r.standard_normal((n, 5)) for _ in range(4)]
    Q = T = None
    full = np.zeros((n, 0))
    for B in blocks:
        Q, T = augment_qr(Q, T, B)
        full = np.hstack([full, B])
        l = full.shape[1]
        np.testing.assert_allclose(Q.T @ Q, np.eye(l), atol=1e-13)
        np.testing.assert_allclose(Q @ T, full, atol=1e-12)
        assert np.allclose(np.tril(T, -1), 0.0)
        assert np.all(np.diag(T) > 0)
    # matches Householder QR of the whole block up to column signs
    Qr, Rr = np.linalg.qr(full)
    sg = np.sign(np.diag(Rr))
    np.testing.assert_allclose(np.abs(T), np.abs(Rr * sg[:, None]), atol=1e-12)


def _exact_rank(m, n, k, seed=0):
    r = np.random.default_rng(seed)
    return r.standard_normal((m, k)) @ r.standard_normal((k, n))


def test_cur_exact_for_exact_rank():
    # rank-k A: CUR-CA with k rows/cols (W nonsingular) reproduces A, so the
    # sketched residual vanishes and rho ~ 0 (skeleton identity)
    m, n, k = 80, 30, 6
    A = _exact_rank(m, n, k)
    S = rng.sparse_sign_matrix(9, 8, m)
    Y = S @ A
    I, J, exh = augment_cur(A, Y, np.zeros(0, int), np.zeros(0, int), None, None, None, k)
    assert len(I) == k and len(J) == k
    C, W, R, E_row = core_and_residual(A, Y, I, J)
    np.testing.assert_allclose(C @ np.linalg.solve(W, R), A, atol=1e-9 * np.abs(A).max())
    assert rho_estimate(E_row, rng.gaussian_probes(9, n, 10)) < 1e-9 * np.linalg.norm(Y)


def test_rho_bounds_spectral_norm():
    r = np.random.default_rng(3)
    for trial in range(20):
        E = r.standard_normal((12, 40)) * (10.0 ** r.uniform(-3, 3))
        rho = rho_estimate(E, rng.gaussian_probes(100 + trial, 40, 10))
        assert rho >= np.linalg.norm(E, 2)


def test_augment_cur_second_step_uses_old_factors():
    # after one step, E_col = A(:,J+) - C W^{-1} R(:,J+) with the old C, W, R:
    # its rows at I are zero (the CUR interpolates A on the selected rows)
    m, n = 60, 25
    A = np.random.default_rng(5).standard_normal((m, n))
    S = rng.sparse_sign_matrix(1, 11, m)
    Y = S @ A
    I, J, _ = augment_cur(A, Y, np.zeros(0, int), np.zeros(0, int), None, None, None, 4)
    C, W, R, E_row = core_and_residual(A, Y, I, J)
    np.testing.assert_allclose(E_row[:, J], 0.0, atol=1e-12)
    I2, J2, _ = augment_cur(A, E_row, I, J, C, W, R, 4)
    assert not set(I2) & set(I) and not set(J2) & set(J)
    Ecol = A[:, J2] - C @ np.linalg.solve(W, R[:, J2])
    np.testing.assert_allclose(Ecol[I, :], 0.0, atol=1e-12)
    # I2 are the LAPACK pivots of E_col with rows I zeroed
    Ecol[I, :] = 0.0
    np.testing.assert_array_equal(I2, lapack_pivots(Ecol, len(J2)))


def _precond_for(A, k, delta, seed=2):
    m, n = A.shape
    S = rng.sparse_sign_matrix(seed, min(m, max(k + 2, int(math.ceil(1.1 * k)))), m)
    Y = S @ A
    I, J, _ = augment_cur(A, Y, np.zeros(0, int), np.zeros(0, int), None, None, None, k)
    C, W, R, E_row = core_and_residual(A, Y, I, J)
    Q, T = augment_qr(None, None, A[I, :].T)
    return Preconditioner(C, W, Q, T, delta), C, W, R


def test_precond_singular_values_of_cur():
    A = np.random.default_rng(7).standard_normal((50, 20))
    P, C, W, R = _precond_for(A, 6, 0.1)
    cur = C @ np.linalg.solve(W, R)
    sv = np.linalg.svd(cur, compute_uv=False)[:6]
    np.testing.assert_allclose(np.sort(P.sigma)[::-1], sv, rtol=1e-10)
    # P^{-1} symmetric, and P P^{-1} = I for the dense P of Alg. 2
    Pi = P.dense_inverse()
    np.testing.assert_allclose(Pi, Pi.T, atol=1e-14)
    V, Lam = P.V, P.Lam
    Pm = V @ np.diag(Lam / P.target) @ V.T + np.eye(20) - V @ V.T
    np.testing.assert_allclose(Pm @ Pi, np.eye(20), atol=1e-12)


def test_two_value_spectrum_exact_rank():
    # exact rank-k A with exact CUR and delta > 0: A_mu P^{-1} has exactly two
    # distinct singular values: the target sqrt(sigma_k^2 + delta^2) (x k) and
    # delta (x n - k), so LSQR converges in two iterations.
    m, n, k, delta = 70, 25, 5, 0.3
    A = _exact_rank(m, n, k, seed=4)
    P, *_ = _precond_for(A, k, delta, seed=8)
    Amu = np.vstack([A, delta * np.eye(n)])
    sv = np.linalg.svd(Amu @ P.dense_inverse(), compute_uv=False)
    np.testing.assert_allclose(sv[:k], P.target, rtol=1e-9)
    np.testing.assert_allclose(sv[k:], delta, rtol=1e-9)
    from oracle.lsqr import plsqr_phase
    b = np.random.default_rng(1).standard_normal(m)
    hist = []
    plsqr_phase(A, delta, b, np.zeros(n), P.inv, eps_lsqr=0.0, tol_ne=0.0, max_iter=3,
                history=hist)
    assert hist[1] <= 1e-12 * max(hist[0], 1.0) or abs(hist[1] - hist[2]) <= 1e-12 * hist[0]


def test_theorem_4_1_bound():
    # kappa(A_mu P^{-1}) <= (sqrt(target^2 + delta^2) + ||E||) / (delta - ||E||)
    r = np.random.default_rng(11)
    m, n, k, delta = 60, 20, 4, 0.5
    A = _exact_rank(m, n, k, seed=6) + 1e-3 * r.standard_normal((m, n))
    P, C, W, R = _precond_for(A, k, delta, seed=3)
    E = A - C @ np.linalg.solve(W, R)
    e = np.linalg.norm(E, 2)
    assert e < delta
    Amu = np.vstack([A, delta * np.eye(n)])
    sv = np.linalg.svd(Amu @ P.dense_inverse(), compute_uv=False)
    assert sv[0] <= math.sqrt(P.target ** 2 + delta ** 2) + e
    assert sv[-1] >= delta - e


def test_sparse_and_dense_paths_agree():
    r = np.random.default_rng(2)
    A = sp.random(200, 40, density=0.2, random_state=3, format="csr")
    Ad = A.toarray()
    S = rng.sparse_sign_matrix(4, 11, 200)
    Ys, Yd = (S @ A).toarray(), S @ Ad
    np.testing.assert_allclose(Ys, Yd, atol=1e-14)
    a = augment_cur(A, Ys, np.zeros(0, int), np.zeros(0, int), None, None, None, 6)
    b = augment_cur(Ad, Yd, np.zeros(0, int), np.zeros(0, int), None, None, None, 6)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


@pytest.mark.parametrize("kappa", [1e6, 1e10, 1e14])
def test_sketched_cholqr_is_the_r_factor(kappa):
    """Sketched Cholesky QR (T_C when chol(C^T C) breaks down): an upper
    triangular T with positive diagonal and T^T T = C^T C to rounding,
    through condition numbers where the plain Cholesky of C^T C fails
    (kappa^2 u > 1), and the same factor as that Cholesky where it exists;
    the rows of C T^{-1} span range(C) with a Gram matrix near I."""
    from oracle.cur import sketched_cholqr
    r = np.random.default_rng(int(np.log10(kappa)))
    m, l = 2500, 150
    U, _ = np.linalg.qr(r.standard_normal((m, l)))
    V, _ = np.linalg.qr(r.standard_normal((l, l)))
    C = (U * np.logspace(0, -np.log10(kappa), l)) @ V.T
    T = sketched_cholqr(C, 5)
    assert T is not None
    assert np.allclose(T, np.triu(T)) and np.all(np.diag(T) > 0)
    assert np.linalg.norm(C.T @ C - T.T @ T) <= 1e-14 * np.linalg.norm(C) ** 2
    Q = np.linalg.solve(T.T, C.T).T
    assert np.linalg.norm(Q.T @ Q - np.eye(l), 2) <= 1e-15 * kappa * 1e2
    try:
        Tc = np.linalg.cholesky(C.T @ C).T
    except np.linalg.LinAlgError:
        assert kappa ** 2 * 2.0 ** -53 > 1.0  # the plain Cholesky fails only past its limit
    else:
        assert np.abs(T - Tc).max() <= 1e-12 * kappa * np.abs(Tc).max()


def test_sketched_cholqr_equals_the_qr_r_factor():
    """Whatever the embedding, T = R' R is the R factor of C: C = (C R^{-1}
    R'^{-1}) (R' R) with an orthonormal first factor and a positive-diagonal
    upper second one, which is unique; T equals numpy's QR factor (signs
    made positive) to rounding (here with k = min(m, 2 l) = m)."""
    from oracle.cur import sketched_cholqr
    r = np.random.default_rng(3)
    C = r.standard_normal((40, 30)) @ np.diag(np.logspace(0, -5, 30))
    T = sketched_cholqr(C, 2)  # k = min(m, 2 l) = 40 = m
    Rq = np.linalg.qr(C)[1]
    Rq = Rq * np.sign(np.diag(Rq))[:, None]
    assert np.abs(T - Rq).max() <= 1e-9 * np.abs(Rq).max()
