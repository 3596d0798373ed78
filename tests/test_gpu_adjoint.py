"""Adjoint of the solve against the oracle (dense QR of the adjoint system,
pinned on the CPU by finite differences) -- GPU tests through the C ABI."""
import numpy as np
import pytest
import torch

from oracle.dense import adjoint, gram_solve, solve_dense_qr
from workloads import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV, dtype=dtype)


def _problem(kind, m, n, k, seed, decades=2.0):
    r = np.random.default_rng(seed)
    if kind == "dense":
        A = synth.dense_svd(r, m, n, 10.0 ** (-decades * np.arange(n) / max(n - 1, 1)))
    else:
        A = synth.sparse_scaled(r, m, n, 6, decades)
    B = r.standard_normal((m, k))
    return A, B


def _gpu(lib, A, dtype=torch.float64):
    if hasattr(A, "tocsr"):
        return lib.CSRMatrix.from_scipy(A, device=DEV, dtype=dtype)
    return _t(A, dtype)


@pytest.mark.parametrize("kind", ["dense", "csr"])
@pytest.mark.parametrize("precond", [False, True])
@pytest.mark.parametrize("k", [1, 3])
def test_backward_matches_oracle(lib, kind, precond, k):
    m, n, mu, tol = 900, 120, 1e-3, 1e-12
    A, B = _problem(kind, m, n, k, 30 + k)
    G = np.random.default_rng(7).standard_normal((n, k))
    with lib.Context(_gpu(lib, A), mu=mu, block=10, tol_ne=tol, precond=precond) as ctx:
        X, info = ctx.solve(_t(B))
        Z, dB, dA, binfo = ctx.solve_backward(X, _t(B), _t(G))
    assert binfo.status == 0 and binfo.eta <= tol * 1.5
    Xn, Zn, dBn = X.cpu().numpy(), Z.cpu().numpy(), dB.cpu().numpy()
    Zr, AZr, dAr = adjoint(A, Xn, B, G, mu)
    scale = np.abs(Zr).max()
    assert np.abs(Zn - Zr).max() <= 1e-8 * scale
    assert np.abs(dBn - AZr).max() <= 1e-8 * np.abs(AZr).max()
    if kind == "dense":
        dAn = dA.cpu().numpy()
        assert np.abs(dAn - dAr).max() <= 1e-8 * np.abs(dAr).max()
    else:
        rows = np.repeat(np.arange(m), np.diff(A.indptr))
        ref = dAr[rows, A.indices]
        assert np.abs(dA.cpu().numpy() - ref).max() <= 1e-8 * np.abs(ref).max()


def test_backward_z_is_gram_solve(lib):
    """Z solves the damped normal equations (second, independent route)."""
    A, B = _problem("dense", 400, 60, 1, 3)
    G = np.random.default_rng(8).standard_normal(60)
    with lib.Context(_t(A), mu=1e-2, tol_ne=1e-13, precond=False) as ctx:
        X, _ = ctx.solve(_t(B[:, 0]))
        Z, dB, dA, info = ctx.solve_backward(X, _t(B[:, 0]), _t(G), want_dA=False)
    assert dA is None
    Zr = gram_solve(A, G, 1e-2)
    assert np.abs(Z.cpu().numpy() - Zr).max() <= 1e-9 * np.abs(Zr).max()


@pytest.mark.parametrize("kind", ["dense", "csr"])
def test_autograd_function(lib, kind):
    """torch.autograd through LstsqFunction: L = sum(X^2) (G = 2 X)."""
    m, n, k, mu = 600, 80, 2, 1e-3
    A, B = _problem(kind, m, n, k, 50)
    Ag = _gpu(lib, A)
    if kind == "dense":
        Ag.requires_grad_(True)
        leaf = Ag
    else:
        Ag.val.requires_grad_(True)
        leaf = Ag.val
    Bg = _t(B).requires_grad_(True)
    X = lib.lstsq_autograd(Ag, Bg, mu=mu, block=8, tol_ne=1e-12)
    loss = (X * X).sum()
    loss.backward()
    Xn = X.detach().cpu().numpy()
    np.testing.assert_allclose(Xn, solve_dense_qr(A, B, mu), rtol=0, atol=1e-8 * np.abs(Xn).max())
    _, AZr, dAr = adjoint(A, Xn, B, 2.0 * Xn, mu)
    np.testing.assert_allclose(Bg.grad.cpu().numpy(), AZr, rtol=0, atol=1e-8 * np.abs(AZr).max())
    if kind == "dense":
        ref = dAr
    else:
        rows = np.repeat(np.arange(m), np.diff(A.indptr))
        ref = dAr[rows, A.indices]
    np.testing.assert_allclose(leaf.grad.cpu().numpy(), ref, rtol=0, atol=1e-8 * np.abs(ref).max())


def test_backward_needs_mu(lib):
    A, B = _problem("dense", 100, 20, 1, 4)
    with lib.Context(_t(A), mu=0.0, precond=False) as ctx:
        X, _ = ctx.solve(_t(B[:, 0]))
        with pytest.raises(lib.AplicurError):
            ctx.solve_backward(X, _t(B[:, 0]), _t(np.ones(20)))
