"""FP32 LSQR phases with FP64 iterative refinement (precision 1): the final
eta is measured in FP64 from a fresh residual, so the FP32 path must reach the
same tolerance and the same solution as the FP64 path and the oracle."""
import numpy as np
import pytest
import torch

from oracle.aplicur import ne_residual
from oracle.dense import solve_dense_qr
from workloads import synth

from bounds import check_solution

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV, dtype=dtype)


@pytest.mark.parametrize("kind", ["dense", "csr"])
@pytest.mark.parametrize("precond", [False, True])
@pytest.mark.parametrize("a_dtype", [torch.float64, torch.float32])
def test_fp32_phases_reach_fp64_tolerance(lib, kind, precond, a_dtype):
    r = np.random.default_rng(60)
    if kind == "dense":
        A = synth.dense_svd(r, 800, 90, 10.0 ** (-4 * np.arange(90) / 89))
    else:
        A = synth.sparse_scaled(r, 5000, 300, 8, 3.0)
    if a_dtype == torch.float32:  # the FP32 values are the problem
        A = A.astype(np.float32).astype(np.float64)
    b = r.standard_normal(A.shape[0])
    mu, tol = 1e-4, 1e-10
    Ag = lib.CSRMatrix.from_scipy(A, device=DEV, dtype=a_dtype) if kind == "csr" else _t(A, a_dtype)
    x, info = lib.lstsq(Ag, _t(b), mu=mu, block=10, tol_ne=tol, precond=precond, precision=1)
    xn = x.cpu().numpy()
    eta = ne_residual(A, b, xn, mu)
    assert info.status == 0
    assert eta <= 1.05 * tol and abs(eta - info.eta) <= 1e-3 * tol
    assert info.phases >= 2  # the FP32 phases alone do not reach 1e-10
    xr = solve_dense_qr(A, b, mu)
    check_solution(xn, xr, A, b, mu, f"FP32 phases {kind} precond={precond} {a_dtype}")


def test_fp32_adjoint(lib):
    r = np.random.default_rng(61)
    A = synth.dense_svd(r, 500, 70, 10.0 ** (-2 * np.arange(70) / 69))
    b = r.standard_normal(500)
    G = r.standard_normal(70)
    mu = 1e-3
    with lib.Context(_t(A), mu=mu, block=8, tol_ne=1e-11, precision=1) as ctx:
        x, _ = ctx.solve(_t(b))
        Z, dB, dA, info = ctx.solve_backward(x, _t(b), _t(G), want_dA=False)
    H = A.T @ A + mu * np.eye(70)
    Zr = np.linalg.solve(H, G)
    assert info.eta <= 1.5e-11
    assert np.abs(Z.cpu().numpy() - Zr).max() <= 1e-7 * np.abs(Zr).max()
