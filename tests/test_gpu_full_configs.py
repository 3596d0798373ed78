"""The workloads at their full sizes, in the launch configuration the
benchmark times.  The small dense one (2000 x 200) is compared with the
oracle's trace and the dense-QR minimiser; the dense kernel and adjoint ones,
which the oracle cannot run, are checked through properties that hold at any
size: every column's normal-equation residual recomputed in FP64 (torch, row
chunks of A widened exactly), and for the adjoint the Gram equation
(A^T A + mu I) Z = G that defines Z and dL/dB = A Z."""
import pytest
import torch

from workloads import synth

pytestmark = pytest.mark.gpu
CHUNK = 8192


def _at(A, R):
    """A^T R in FP64 over row chunks of the FP32 A."""
    out = torch.zeros(A.shape[1], R.shape[1], dtype=torch.float64, device=A.device)
    for i0 in range(0, A.shape[0], CHUNK):
        out += A[i0:i0 + CHUNK].to(torch.float64).T @ R[i0:i0 + CHUNK]
    return out


def _a(A, X):
    """A X in FP64 over row chunks of the FP32 A."""
    return torch.cat([A[i0:i0 + CHUNK].to(torch.float64) @ X for i0 in range(0, A.shape[0], CHUNK)])


def _eta(A, B, X, mu):
    N = _at(A, B - _a(A, X)) - mu * X
    return N.norm(dim=0) / _at(A, B).norm(dim=0)


@pytest.fixture(scope="module")
def kernel_workload():
    # Gaussian RBF kernel (h = 1) on 40000 points in [0,1]^8, FP32 A, 16 RHS
    A, B = synth.rbf_kernel_gpu(3003, 40000, 16)
    yield A, B
    del A, B
    torch.cuda.empty_cache()


@pytest.mark.parametrize("precision", [0, 2])
def test_kernel_workload_full_size(lib, kernel_workload, precision):
    A, B = kernel_workload
    mu = 1e-3
    X, info = lib.lstsq(A, B, mu=mu, block=250, tol_ne=1e-8, precision=precision)
    eta = _eta(A, B, X, mu)
    assert info.status == 0
    assert float(eta.max()) <= 1.05e-8
    assert abs(float(eta.max()) - info.eta) <= 1e-2 * 1e-8


def test_adjoint_workload_full_size(lib):
    # dense FP32 100000 x 2000, sigma_i = 10^(-5 i / 2000), 32 RHS, L = sum X^2
    A, B = synth.dense_svd_gpu(5000, 100000, 2000, 5.0, 32)
    mu, tol = 1e-5, 1e-8
    with lib.Context(A, mu=mu, block=100, tol_ne=tol) as ctx:
        X, info = ctx.solve(B)
        G = 2.0 * X
        Z, dB, _, binfo = ctx.solve_backward(X, B, G, want_dA=False)
    assert info.status == 0 and binfo.status == 0
    assert float(_eta(A, B, X, mu).max()) <= 1.05 * tol
    # Z solves min || A_mu Z - [0; G / delta] ||: its normal equations are
    # (A^T A + mu I) Z = G, relative to ||A_mu^T [0; G / delta]|| = ||G||
    AZ = _a(A, Z)
    res = (_at(A, AZ) + mu * Z - G).norm(dim=0) / G.norm(dim=0)
    assert float(res.max()) <= 1.05 * tol
    assert float((dB - AZ).norm() / AZ.norm()) <= 1e-12
    del A, B, X, Z, dB, AZ
    torch.cuda.empty_cache()


def test_small_dense_workload_full_size(lib):
    """Dense FP64 2000 x 200, sigma_i = 10^(-6 i / 200), mu = 0, tol 1e-10: at
    full size the oracle runs too, so the CUR sequence is compared with its
    trace and the solution with the dense-QR minimiser."""
    import numpy as np

    from oracle.aplicur import Options, Trace, aplicur, ne_residual
    from oracle.dense import solve_dense_qr

    w = synth.workload(1, 1.0)
    tr = Trace()
    aplicur(w.A, w.B, 0.0, Options(block=w.block, tol_ne=w.tol), tr)
    At = torch.as_tensor(w.A, device="cuda")
    with lib.Context(At, mu=0.0, block=w.block, tol_ne=w.tol) as ctx:
        x, info = ctx.solve(torch.as_tensor(w.B, device="cuda"))
        ranks = ctx.query(8).tolist()
    x = x.cpu().numpy()
    eta = ne_residual(w.A, w.B, x, 0.0)
    assert info.status == 0 and eta <= 1.05 * w.tol
    k = min(len(ranks), len(tr.ranks))
    assert abs(len(ranks) - len(tr.ranks)) <= 1 and ranks[:k] == tr.ranks[:k]
    xr = solve_dense_qr(w.A, w.B, 0.0)
    smin = np.linalg.svd(w.A, compute_uv=False)[-1]
    bound = eta * np.linalg.norm(w.A.T @ w.B) / smin ** 2
    assert np.linalg.norm(x - xr) <= 2 * bound + 1e-9 * np.linalg.norm(xr)
