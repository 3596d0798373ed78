"""Blocked multi-right-hand-side path (dense A, several columns through the
MFMA products) against the oracle -- GPU tests through the C ABI.

Products are checked element by element against the FP64 CPU product; solves
per column against the dense-QR oracle, through the normal-equation residual
recomputed on the CPU and the error bound it implies:
||x - x*|| <= eta ||A^T b|| / lambda_min(A^T A + mu I)."""
import numpy as np
import pytest
import torch

from oracle.aplicur import ne_residual
from oracle.dense import adjoint, solve_dense_qr
from workloads import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV, dtype=dtype)


def _dense(m, n, seed, decades=3.0):
    r = np.random.default_rng(seed)
    return synth.dense_svd(r, m, n, 10.0 ** (-decades * np.arange(n) / max(n - 1, 1)))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("m,n,k,pad", [(1000, 237, 5, 0), (333, 1025, 16, 0), (1201, 64, 17, 3),
                                       (130, 2050, 40, 1), (517, 129, 70, 0)])
def test_matmat_matches_cpu(lib, dtype, m, n, k, pad):
    """A X and A^T X (ragged m, n; k across the 16/32/64 column blocks and
    two groups; pad > 0: a leading dimension that rules out vector loads)."""
    r = np.random.default_rng(m + n + k)
    A = r.standard_normal((m, n)) * np.exp(r.uniform(-2, 2, (m, n)))
    if dtype == torch.float32:
        A = A.astype(np.float32).astype(np.float64)
    big = torch.zeros((m, n + pad), device=DEV, dtype=dtype)
    big[:, :n] = _t(A, dtype)
    Ag = big[:, :n]
    X, U = r.standard_normal((n, k)), r.standard_normal((m, k))
    with lib.Context(Ag, mu=1e-3, precond=False) as ctx:
        Y = ctx.matmat(_t(X)).cpu().numpy()
        Z = ctx.matmat(_t(U), trans=True).cpu().numpy()
    # elementwise bound of any summation order: |fl(sum) - sum| <= gamma_len sum |terms|
    absA = np.abs(A)
    assert np.all(np.abs(Y - A @ X) <= (n + 2) * 1.2e-16 * (absA @ np.abs(X)))
    assert np.all(np.abs(Z - A.T @ U) <= (m + 2) * 1.2e-16 * (absA.T @ np.abs(U)))


def _check_columns(A, B, X, mu, tol, slack=1.05):
    """Every column: eta (oracle metric) <= slack tol, and the error bound."""
    n = A.shape[1]
    lam = np.linalg.eigvalsh(A.T @ A + mu * np.eye(n))[0]
    Xr = solve_dense_qr(A, B, mu)
    for j in range(B.shape[1]):
        eta = ne_residual(A, B[:, j], X[:, j], mu)
        assert eta <= slack * tol, (j, eta)
        bound = eta * np.linalg.norm(A.T @ B[:, j]) / lam
        assert np.linalg.norm(X[:, j] - Xr[:, j]) <= 1.1 * bound + 1e-12 * np.linalg.norm(Xr[:, j]), j


@pytest.mark.parametrize("precond", [False, True])
@pytest.mark.parametrize("k", [2, 5, 20, 70])
def test_blocked_solve_matches_oracle(lib, precond, k):
    m, n, mu, tol = 700, 90, 1e-6, 1e-10
    A = _dense(m, n, 40 + k, decades=4)
    B = np.random.default_rng(k).standard_normal((m, k))
    X, info = lib.lstsq(_t(A), _t(B), mu=mu, block=10, tol_ne=tol, precond=precond)
    assert info.status == 0 and info.eta <= tol
    _check_columns(A, B, X.cpu().numpy(), mu, tol)


def test_product_kernel_event_timing(lib):
    """aplicur_prof_products / aplicur_prof_read: with timing on, a blocked
    solve's A X and A^T U launches are recorded with positive durations and
    the solution is unchanged; off, nothing more is recorded."""
    m, n, mu, tol = 700, 90, 1e-6, 1e-10
    A = _dense(m, n, 44, decades=4)
    B = np.random.default_rng(3).standard_normal((m, 4))
    X0, _ = lib.lstsq(_t(A), _t(B), mu=mu, block=10, tol_ne=tol)
    lib.prof_read()
    lib.prof_products(True)
    try:
        X1, info = lib.lstsq(_t(A), _t(B), mu=mu, block=10, tol_ne=tol)
        rec = lib.prof_read()
    finally:
        lib.prof_products(False)
    print(f"[prof] {rec}")
    assert torch.equal(X0, X1)
    for kind in ("AX_f64", "ATX_f64"):
        launches, mean_us, untimed = rec[kind]
        assert launches >= info.iters and mean_us > 0.0 and untimed == 0
    lib.lstsq(_t(A), _t(B), mu=mu, block=10, tol_ne=tol)
    assert lib.prof_read() == {}


def test_blocked_fp32_values_mu_zero(lib):
    """FP32 A (values widened exactly), mu = 0 (m > n), APLICUR."""
    m, n, tol = 800, 70, 1e-10
    A = _dense(m, n, 51, decades=3).astype(np.float32).astype(np.float64)
    B = np.random.default_rng(52).standard_normal((m, 6))
    X, info = lib.lstsq(_t(A, torch.float32), _t(B), mu=0.0, block=8, tol_ne=tol)
    assert info.status == 0
    _check_columns(A, B, X.cpu().numpy(), 0.0, tol)


def test_blocked_matches_columns_one_at_a_time(lib):
    """Columns solved together reach the solutions of one-at-a-time solves
    (both to the solve's accuracy) with similar iteration counts."""
    m, n, mu, tol = 300, 40, 1e-5, 1e-10
    A = _dense(m, n, 18, decades=4)
    B = np.random.default_rng(4).standard_normal((m, 3))
    X, info = lib.lstsq(_t(A), _t(B), mu=mu, block=6, tol_ne=tol)
    X = X.cpu().numpy()
    its = []
    for j in range(3):
        xj, inf = lib.lstsq(_t(A), _t(B[:, j]), mu=mu, block=6, tol_ne=tol)
        its.append(inf.iters)
        scale = np.linalg.norm(xj.cpu().numpy())
        assert np.linalg.norm(X[:, j] - xj.cpu().numpy()) <= 1e-6 * scale
    assert abs(info.iters - max(its)) <= max(3, 0.1 * max(its))


def test_columns_option_is_columnwise(lib):
    """columns=1: the column path, bitwise equal to one-at-a-time solves."""
    A = _dense(300, 40, 18, decades=4)
    B = np.random.default_rng(4).standard_normal((300, 3))
    X, info = lib.lstsq(_t(A), _t(B), mu=1e-5, block=6, tol_ne=1e-10, columns=1)
    X = X.cpu().numpy()
    for k in range(3):
        xk, _ = lib.lstsq(_t(A), _t(B[:, k]), mu=1e-5, block=6, tol_ne=1e-10)
        assert np.array_equal(X[:, k], xk.cpu().numpy())


def test_blocked_zero_column_and_warm_start(lib):
    m, n, mu, tol = 400, 50, 1e-4, 1e-11
    A = _dense(m, n, 61)
    B = np.random.default_rng(62).standard_normal((m, 4))
    B[:, 2] = 0.0
    Ag = _t(A)
    with lib.Context(Ag, mu=mu, block=6, tol_ne=tol) as ctx:
        X, info = ctx.solve(_t(B))
        Xn = X.cpu().numpy()
        assert np.all(Xn[:, 2] == 0.0)
        _check_columns(A, B, Xn, mu, tol)
        # warm start from the exact solution: no further work beyond the checks
        Xr = solve_dense_qr(A, B, mu)
        X1, info1 = ctx.solve(_t(B), X0=_t(Xr))
        assert info1.iters <= 5
        _check_columns(A, B, X1.cpu().numpy(), mu, tol)


@pytest.mark.parametrize("precond", [False, True])
def test_blocked_adjoint_matches_oracle(lib, precond):
    m, n, k, mu, tol = 900, 120, 7, 1e-3, 1e-12
    r = np.random.default_rng(71)
    A = synth.dense_svd(r, m, n, 10.0 ** (-2.0 * np.arange(n) / (n - 1)))
    B = r.standard_normal((m, k))
    G = r.standard_normal((n, k))
    with lib.Context(_t(A), mu=mu, block=10, tol_ne=tol, precond=precond) as ctx:
        X, info = ctx.solve(_t(B))
        Z, dB, dA, binfo = ctx.solve_backward(X, _t(B), _t(G))
    assert binfo.status == 0 and binfo.eta <= tol * 1.5
    Zr, AZr, dAr = adjoint(A, X.cpu().numpy(), B, G, mu)
    assert np.abs(Z.cpu().numpy() - Zr).max() <= 1e-8 * np.abs(Zr).max()
    assert np.abs(dB.cpu().numpy() - AZr).max() <= 1e-8 * np.abs(AZr).max()
    assert np.abs(dA.cpu().numpy() - dAr).max() <= 1e-8 * np.abs(dAr).max()


@pytest.mark.parametrize("a_dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("precond", [False, True])
@pytest.mark.parametrize("mu", [1e-4, 0.0])
def test_blocked_fp32_phases_reach_fp64_tolerance(lib, a_dtype, precond, mu):
    """Precision 1 with several columns: FP32 blocked phases (FP32 MFMA
    products) and FP64 refinement reach the FP64 tolerance per column."""
    m, n, tol = 800, 90, 1e-10
    A = _dense(m, n, 60, decades=4)
    if a_dtype == torch.float32:  # the FP32 values are the problem
        A = A.astype(np.float32).astype(np.float64)
    B = np.random.default_rng(61).standard_normal((m, 5))
    X, info = lib.lstsq(_t(A, a_dtype), _t(B), mu=mu, block=10, tol_ne=tol, precond=precond, precision=1)
    assert info.status == 0
    assert info.phases >= 2  # the FP32 phases alone do not reach 1e-10
    _check_columns(A, B, X.cpu().numpy(), mu, tol)


def test_blocked_fp32_adjoint(lib):
    r = np.random.default_rng(62)
    A = synth.dense_svd(r, 500, 70, 10.0 ** (-2 * np.arange(70) / 69))
    B = r.standard_normal((500, 4))
    G = r.standard_normal((70, 4))
    mu = 1e-3
    with lib.Context(_t(A), mu=mu, block=8, tol_ne=1e-11, precision=1) as ctx:
        X, _ = ctx.solve(_t(B))
        Z, dB, dA, info = ctx.solve_backward(X, _t(B), _t(G), want_dA=False)
    Zr = np.linalg.solve(A.T @ A + mu * np.eye(70), G)
    assert info.eta <= 1.5e-11
    assert np.abs(Z.cpu().numpy() - Zr).max() <= 1e-7 * np.abs(Zr).max()


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_blocked_kernel_workload_half_size(lib, precision):
    """The configuration bench.py times for several right-hand sides (RBF
    kernel on 20000 points, FP32 A, 16 RHS, mu = 1e-3, block 250): every
    column's eta recomputed on the CPU in FP64 from the FP32 values."""
    A, B = synth.rbf_kernel_gpu(3003, 20000, 16)
    tol, mu = 1e-8, 1e-3
    X, info = lib.lstsq(A, B, mu=mu, block=250, tol_ne=tol, precision=precision)
    assert info.status == 0
    An = A.cpu().numpy().astype(np.float64)
    Bn, Xn = B.cpu().numpy(), X.cpu().numpy()
    R = Bn - An @ Xn
    N = An.T @ R - mu * Xn
    atb = np.linalg.norm(An.T @ Bn, axis=0)
    eta = np.linalg.norm(N, axis=0) / atb
    assert np.all(eta <= 1.05 * tol), eta
    assert abs(eta.max() - info.eta) <= 1e-2 * tol


def _bf16(a):
    """Round-to-nearest-even BF16 values of an FP32 array, widened to FP64."""
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


@pytest.mark.parametrize("prec", [1, 2])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("m,n,k,pad", [(1000, 237, 5, 0), (333, 1025, 16, 0), (1201, 64, 17, 3),
                                       (130, 2050, 40, 1), (517, 129, 70, 0)])
def test_matmat_low_precision_products(lib, prec, dtype, m, n, k, pad):
    """The FP32 (prec 1) and BF16 (prec 2) products of the low-precision
    phases against the FP64 product of the rounded operands: X rounded to
    FP32, A to FP32 (and to BF16 for prec 2; the tiles pad rows to 32 and
    columns to 64).  Bound per entry: FP32 accumulation over the reduction
    length plus the S plane sums, gamma_(len+64) with u = 2^-24, and for prec
    2 the two-part BF16 split of X (|x - hi - lo| <= 2^-18 |x|)."""
    r = np.random.default_rng(m + n + k + 7 * prec)
    A = r.standard_normal((m, n)) * np.exp(r.uniform(-2, 2, (m, n)))
    big = torch.zeros((m, n + pad), device=DEV, dtype=dtype)
    big[:, :n] = _t(A, dtype)
    A32 = A.astype(np.float32).astype(np.float64)
    Aq = _bf16(A32) if prec == 2 else A32
    X, U = r.standard_normal((n, k)), r.standard_normal((m, k))
    X32, U32 = X.astype(np.float32).astype(np.float64), U.astype(np.float32).astype(np.float64)
    with lib.Context(big[:, :n], mu=1e-3, precond=False, precision=prec) as ctx:
        Y = ctx.matmat(_t(X), prec=prec).cpu().numpy()
        Z = ctx.matmat(_t(U), trans=True, prec=prec).cpu().numpy()
    split = 2.0 ** -18 if prec == 2 else 0.0
    u = 2.0 ** -24
    ref_y, ref_z = Aq @ X32, Aq.T @ U32
    abs_y, abs_z = np.abs(Aq) @ np.abs(X32), np.abs(Aq).T @ np.abs(U32)
    assert np.all(np.abs(Y - ref_y) <= ((n + 64) * u + split) * abs_y)
    assert np.all(np.abs(Z - ref_z) <= ((m + 64) * u + split) * abs_z)
    if prec == 2:  # the BF16 rounding of A is really there
        assert np.abs(Y - A32 @ X32).max() > 10 * np.abs(Y - ref_y).max()


def test_matmat_prec_needs_the_operator(lib):
    A = _t(_dense(200, 40, 3))
    with lib.Context(A, mu=1e-3, precond=False) as ctx:
        with pytest.raises(RuntimeError, match="prec 1"):
            ctx.matmat(_t(np.ones((40, 2))), prec=1)
    with lib.Context(A, mu=1e-3, precond=False, precision=1) as ctx:
        with pytest.raises(RuntimeError, match="prec 2"):
            ctx.matmat(_t(np.ones((40, 2))), prec=2)


@pytest.mark.parametrize("a_dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("precond", [False, True])
@pytest.mark.parametrize("mu", [1e-4, 0.0])
def test_blocked_bf16_phases_reach_fp64_tolerance(lib, a_dtype, precond, mu):
    """Precision 2: BF16 products in the low-precision phases, FP32 products
    once a BF16 phase gains too little, FP64 refinement: every column reaches
    the FP64 tolerance."""
    m, n, tol = 800, 90, 1e-10
    A = _dense(m, n, 60, decades=4)
    if a_dtype == torch.float32:
        A = A.astype(np.float32).astype(np.float64)
    B = np.random.default_rng(61).standard_normal((m, 5))
    X, info = lib.lstsq(_t(A, a_dtype), _t(B), mu=mu, block=10, tol_ne=tol, precond=precond, precision=2)
    assert info.status == 0
    assert info.phases_bf16 >= 1
    _check_columns(A, B, X.cpu().numpy(), mu, tol)


def test_blocked_bf16_well_conditioned_stays_bf16(lib):
    """A well-conditioned problem: the BF16 phases divide eta by more than 10
    each, so the ladder keeps them; the FP64 tolerance is still reached."""
    m, n, mu, tol = 1500, 100, 1e-2, 1e-10
    A = _dense(m, n, 64, decades=0.5)
    B = np.random.default_rng(65).standard_normal((m, 3))
    X, info = lib.lstsq(_t(A), _t(B), mu=mu, tol_ne=tol, precond=False, precision=2)
    assert info.status == 0
    assert info.phases_bf16 == info.phases
    _check_columns(A, B, X.cpu().numpy(), mu, tol)


def test_blocked_bf16_adjoint(lib):
    r = np.random.default_rng(66)
    A = synth.dense_svd(r, 500, 70, 10.0 ** (-2 * np.arange(70) / 69))
    B = r.standard_normal((500, 4))
    G = r.standard_normal((70, 4))
    mu = 1e-3
    with lib.Context(_t(A), mu=mu, block=8, tol_ne=1e-11, precision=2) as ctx:
        X, _ = ctx.solve(_t(B))
        Z, dB, dA, info = ctx.solve_backward(X, _t(B), _t(G), want_dA=False)
    Zr = np.linalg.solve(A.T @ A + mu * np.eye(70), G)
    assert info.eta <= 1.5e-11
    assert np.abs(Z.cpu().numpy() - Zr).max() <= 1e-7 * np.abs(Zr).max()
