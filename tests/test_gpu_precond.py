"""Parity of the set-up at the block sizes of the benchmark workloads, and of
the preconditioner itself (not only through the solutions it produces).

* Alg. 7 / Alg. 3 Part 1 at b = 50 and b = 100: the library's blocked pivot
  search takes 32 pivots per panel with a trailing update, and its Schur-block
  inverse and Cholesky factors take 64-column panels; these sizes cross both.
  The CUR indices I, J must equal the oracle's bit for bit over three outer
  steps, and rho must agree to 1e-9 relative.
* Sec. 5.1: the sketch Y = S A at s = 110 and s = 275 (blocks 100 and 250).
* Alg. 2 Part 2: the core singular values of the one-sided Jacobi SVD against
  the oracle's LAPACK SVD, within the bound its stopping test gives: with E
  the scaled off-diagonal of the damped core's Gram matrix in the Jacobi
  basis, the exact values Lambda_k^2 = sigma_k^2 + delta^2 equal theta_k times
  the Jacobi ones with theta_k in [1 - ||E||_2, 1 + ||E||_2] (Ostrowski), and
  ||E||_2 <= ||E||_F <= jacobi_tol.
* P^{-1} z and P^{-T} z element by element against the oracle's
  Preconditioner / SvdFreePreconditioner built from the same I, J, with the
  Jacobi sweeps run to convergence (P depends on M only, so the SVD's sign
  and order conventions do not matter): within 1e-10 of ||P^{-1}|| ||z||.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import torch

from oracle import rng as orng
from oracle.aplicur import Options, Trace, aplicur, sketch_rows
from oracle.cur import Preconditioner, SvdFreePreconditioner
from workloads import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV, dtype=dtype)


def _problem(kind, m, n, seed, decades):
    r = np.random.default_rng(seed)
    if kind == "dense":
        sigma = 10.0 ** (-decades * np.arange(n) / max(n - 1, 1))
        return synth.dense_svd(r, m, n, sigma)
    return synth.sparse_scaled(r, m, n, 10, decades)


def _gpu(lib, A):
    if sp.issparse(A):
        return lib.CSRMatrix.from_scipy(A, device=DEV)
    return _t(A)


def _dense(A):
    return A.toarray() if sp.issparse(A) else A


def _qr_pos(Rt):
    Q, T = np.linalg.qr(Rt)
    sg = np.where(np.diag(T) < 0, -1.0, 1.0)
    return Q * sg, T * sg[:, None]


# ----------------------------------------------------------------- Alg. 7 at the benchmark block sizes
@pytest.mark.parametrize("kind", ["dense", "csr"])
@pytest.mark.parametrize("block", [50, 100])
def test_cur_indices_at_benchmark_block_sizes(lib, kind, block):
    A = _problem(kind, 3000, 450, 40 + block, 3.0)
    b = np.random.default_rng(7).standard_normal(A.shape[0])
    mu, seed, steps = 1e-8, 9, 3
    # the fixed-rank schedule builds P only at the cap, so the CUR sequence
    # runs its three steps with no LSQR phase in between (the sequence itself
    # does not depend on the schedule)
    tr = Trace()
    aplicur(A, b, mu, Options(block=block, seed=seed, tol_ne=1e-30, max_rank=block * steps, max_iter=3,
                              schedule=2), tr)
    with lib.Context(_gpu(lib, A), mu=mu, block=block, seed=seed, tol_ne=1e-30, max_rank=block * steps,
                     max_iter=3, schedule=2) as ctx:
        ctx.solve(_t(b))
        ranks, rhos = ctx.query(8), ctx.query(7)
        I, J = ctx.query(6), ctx.query(5)
    print(f"[parity] {kind} b={block}: ranks {list(ranks)}, rho {rhos}")
    assert list(ranks) == tr.ranks[:len(ranks)] and len(ranks) == steps
    np.testing.assert_array_equal(J, tr.J[:len(J)])
    np.testing.assert_array_equal(I, tr.I[:len(I)])
    np.testing.assert_allclose(rhos, tr.rhos[:len(rhos)], rtol=1e-9)


@pytest.mark.parametrize("kind", ["dense", "csr"])
@pytest.mark.parametrize("block", [100, 250])
def test_sketch_at_benchmark_sizes(lib, kind, block):
    m, n, seed = 6000, 700, 12
    A = _problem(kind, m, n, 3, 2.0)
    with lib.Context(_gpu(lib, A), mu=1e-4, block=block, seed=seed, max_outer=1, max_iter=1) as ctx:
        s = ctx.sizes()["s"]
        assert s == sketch_rows(block, m) == round(1.1 * block)
        Y = ctx.query(1).reshape(s, n)
        rows, signs = ctx.query(2).reshape(m, 8), ctx.query(3).reshape(m, 8)
    r_or, s_or, _ = orng.sparse_sign(seed, s, m, 8)
    np.testing.assert_array_equal(rows, r_or)
    np.testing.assert_array_equal(signs, s_or)
    S = orng.sparse_sign_matrix(seed, s, m, 8)
    Yref = np.asarray(S @ _dense(A))
    # every entry of Y is a sum of at most m terms |S_hi a_ij| in FP64
    mag = np.asarray(abs(S) @ np.abs(_dense(A)))
    err = np.abs(Y - Yref).max()
    print(f"[parity] sketch {kind} s={s}: max |Y - S A| = {err:.3e} (max |Y| {np.abs(Yref).max():.3e})")
    assert np.all(np.abs(Y - Yref) <= 1e-13 * mag + 1e-300)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_dense_sketch_equals_csr_sketch(lib, dtype):
    """Both sketch kernels sum each entry of Y over the rows of A in
    increasing order, each term the rounded +-a/sqrt(xi): the dense sketch of
    a matrix with no zero entries equals the CSR sketch of the same matrix bit
    for bit (ragged sizes: n not a multiple of the 256-column strip, m not a
    multiple of the 256-row chunk of the inverse map)."""
    m, n, block, seed = 5003, 517, 60, 4
    A = np.random.default_rng(2).standard_normal((m, n))
    assert np.all(A != 0)
    Ys = []
    for Ag in (_t(A, dtype), lib.CSRMatrix.from_scipy(sp.csr_matrix(A), device=DEV, dtype=dtype)):
        with lib.Context(Ag, mu=1e-4, block=block, seed=seed, max_outer=1, max_iter=1) as ctx:
            s = ctx.sizes()["s"]
            Ys.append(ctx.query(1).reshape(s, n))
    print(f"[parity] dense vs CSR sketch {dtype}: max |diff| {np.abs(Ys[0] - Ys[1]).max():.3e}")
    np.testing.assert_array_equal(Ys[0], Ys[1])


# ----------------------------------------------------------------- Alg. 2: the core SVD and P itself
def _oracle_factors(A, I, J):
    C = A[:, J]
    W = _dense(A[I, :][:, J]) if sp.issparse(A) else A[np.ix_(I, J)]
    Q, T = _qr_pos(_dense(A[I, :]).T)
    return C, W, Q, T


@pytest.mark.parametrize("kind", ["dense", "csr"])
def test_jacobi_singular_values_within_their_bound(lib, kind):
    """Default stopping level 1e-2: the Jacobi core singular values (query
    11) against the oracle's SVD of the same core."""
    A = _problem(kind, 1500 if kind == "dense" else 6000, 160, 50, 6.0)
    b = np.random.default_rng(8).standard_normal(A.shape[0])
    mu, block, tol_j = 1e-6, 20, 1e-2
    with lib.Context(_gpu(lib, A), mu=mu, block=block, tol_ne=1e-10) as ctx:
        ctx.solve(_t(b))
        sig = np.sort(ctx.query(11))[::-1]
        I, J = ctx.query(6), ctx.query(5)
        sweeps = ctx.query(14)
    P = Preconditioner(*_oracle_factors(A, I, J), math.sqrt(mu))
    assert len(sig) == len(P.sigma) == len(I)
    lam_gpu = sig ** 2 + mu
    lam_or = P.sigma ** 2 + mu
    ratio = lam_or / lam_gpu
    print(f"[parity] Jacobi {kind}: rank {len(I)}, sweeps {list(sweeps)}, "
          f"Lambda^2 ratio in [{ratio.min():.6f}, {ratio.max():.6f}]")
    slack = 1e-10
    assert ratio.min() >= 1.0 - tol_j - slack and ratio.max() <= 1.0 + tol_j + slack


def test_precond_apply_after_blocked_solve(lib):
    """With several right-hand sides of a dense A the library applies P as
    z + Q_R W Q_R^T z (W = V_M diag(d) V_M^T) and never forms V = Q_R V_M;
    a one-column P-apply on the same build forms V then, and the blocked
    form is restored for the adjoint solve after it.  P^{-1} z must match the
    oracle (as in the one-column case below), and the adjoint's dB must equal,
    bit for bit, that of a run without the P-apply in between."""
    A = _problem("dense", 1200, 120, 51, 2.0)
    B = np.random.default_rng(9).standard_normal((A.shape[0], 3))
    G = np.random.default_rng(11).standard_normal((A.shape[1], 3))
    z = np.random.default_rng(10).standard_normal(A.shape[1])
    mu, block = 1e-4, 10

    def run(apply_between):
        with lib.Context(_gpu(lib, A), mu=mu, block=block, tol_ne=1e-10, jacobi_tol=1e-15) as ctx:
            X, info = ctx.solve(_t(B))
            assert info.status == 0
            I, J = ctx.query(6), ctx.query(5)
            y = ctx.precond_apply(_t(z)).cpu().numpy() if apply_between else None
            _, dB, _, binfo = ctx.solve_backward(X, _t(B), _t(G), want_dA=False)
            assert binfo.status == 0
            return I, J, y, dB.cpu().numpy()

    I, J, y, dB1 = run(True)
    I0, J0, _, dB0 = run(False)
    np.testing.assert_array_equal(I, I0)
    np.testing.assert_array_equal(J, J0)
    P = Preconditioner(*_oracle_factors(A, I, J), math.sqrt(mu))
    err = np.abs(y - P.inv(z)).max()
    print(f"[parity] P^-1 z after a blocked solve: rank {len(I)}, max error {err:.3e} (||z|| {np.linalg.norm(z):.3e})")
    assert err <= 1e-10 * np.linalg.norm(z)
    np.testing.assert_array_equal(dB1, dB0)


@pytest.mark.parametrize("kind", ["dense", "csr"])
def test_precond_apply_matches_oracle(lib, kind):
    """P^{-1} z (symmetric: P^{-T} z too) element by element, Jacobi run to
    convergence."""
    A = _problem(kind, 1200 if kind == "dense" else 5000, 120, 51, 2.0)
    b = np.random.default_rng(9).standard_normal(A.shape[0])
    mu, block = 1e-4, 10
    with lib.Context(_gpu(lib, A), mu=mu, block=block, tol_ne=1e-10, jacobi_tol=1e-15) as ctx:
        ctx.solve(_t(b))
        I, J = ctx.query(6), ctx.query(5)
        z = np.random.default_rng(10).standard_normal(A.shape[1])
        y = ctx.precond_apply(_t(z)).cpu().numpy()
        yt = ctx.precond_apply(_t(z), trans=True).cpu().numpy()
    P = Preconditioner(*_oracle_factors(A, I, J), math.sqrt(mu))
    yr = P.inv(z)
    scale = np.linalg.norm(z)  # ||P^{-1}||_2 <= 1 (sigma_hat <= Lambda_i)
    err = max(np.abs(y - yr).max(), np.abs(yt - yr).max())
    print(f"[parity] P^-1 z {kind}: rank {len(I)}, max error {err:.3e} (||z|| {scale:.3e})")
    assert err <= 1e-10 * scale


@pytest.mark.parametrize("kind,cap", [("dense", 0), ("csr", 0), ("csr", 60)])
def test_svdfree_apply_matches_oracle(lib, kind, cap):
    """Alg. 8 (mu = 0): P~^{-1} z and P~^{-T} z element by element against
    the oracle's SvdFreePreconditioner from the same I, J and target level;
    full rank, and a rank cap that leaves I - Q_R Q_R^T in play."""
    A = _problem(kind, 1200 if kind == "dense" else 5000, 120, 52, 2.0)
    b = np.random.default_rng(11).standard_normal(A.shape[0])
    block = 10
    tr = Trace()
    aplicur(A, b, 0.0, Options(block=block, tol_ne=1e-10, max_rank=cap, precond="svdfree"), tr)
    with lib.Context(_gpu(lib, A), mu=0.0, block=block, tol_ne=1e-10, max_rank=cap, precond="svdfree") as ctx:
        ctx.solve(_t(b))
        I, J = ctx.query(6), ctx.query(5)
        rhos = ctx.query(7)
        z = np.random.default_rng(12).standard_normal(A.shape[1])
        y = ctx.precond_apply(_t(z)).cpu().numpy()
        yt = ctx.precond_apply(_t(z), trans=True).cpu().numpy()
    np.testing.assert_array_equal(J, tr.J)
    np.testing.assert_array_equal(I, tr.I)
    eps_cur = 3e-7  # the mu = 0 reading of eps_cur
    P = SvdFreePreconditioner(*_oracle_factors(A, I, J), tr.rhos[-1], eps_cur)
    assert abs(max(rhos[-1], eps_cur) - P.target) <= 1e-9 * P.target
    yr, ytr = P.inv(z), P.inv_t(z)
    # the apply forms z + Q_R (H (Q_R^T z)), H = t M^{-1} - I: its rounding is
    # relative to ||z|| (1 + ||H||), whatever the size of the result (at full
    # rank z - Q_R Q_R^T z cancels)
    H = P.target * P.Minv - np.eye(P.Minv.shape[0])
    scale = (np.linalg.norm(P.dense_inverse(), 2) + 1.0 + np.linalg.norm(H, 2)) * np.linalg.norm(z)
    err = max(np.abs(y - yr).max(), np.abs(yt - ytr).max())
    print(f"[parity] P~^-1 z {kind} cap {cap}: rank {len(I)}, max error {err:.3e} (scale {scale:.3e})")
    assert err <= 1e-10 * scale
    # the two applies differ (P~ is not symmetric), so the test tells them apart
    assert np.abs(yr - ytr).max() > 1e-3 * np.abs(yr).max()
