"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances: FP64 element-wise results 1e-10 relative to the operand norms
(the stated FP64 bar); solutions within the conditioning bound of the
normal-equation residual they reach (tests/bounds.py); integer / index
results bit-exact.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import torch

from oracle import rng as orng
from oracle.aplicur import Options, Trace, aplicur, lsqr_plain, ne_residual
from oracle.cur import augment_cur, core_and_residual, rho_estimate
from oracle.dense import solve_dense_qr
from oracle.lsqr import plsqr_phase
from workloads import synth

from bounds import check_solution

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV, dtype=dtype)


def _dense(m, n, seed, decades=3.0):
    r = np.random.default_rng(seed)
    sigma = 10.0 ** (-decades * np.arange(n) / max(n - 1, 1))
    return synth.dense_svd(r, m, n, sigma)


def _csr(m, n, per_row, seed, decades=2.0):
    return synth.sparse_scaled(np.random.default_rng(seed), m, n, per_row, decades)


def _gpu_csr(A, dtype=torch.float64):
    import paper_2604_05065_amd as ap
    return ap.CSRMatrix.from_scipy(A, device=DEV, dtype=dtype)


# ----------------------------------------------------------------- sketch
@pytest.mark.parametrize("kind,m,n,block", [("dense", 300, 37, 6), ("dense", 1000, 130, 20),
                                             ("csr", 2000, 300, 10), ("csr", 513, 64, 3)])
def test_sketch_matches_oracle(lib, kind, m, n, block, xi=8):
    seed = 11
    if kind == "dense":
        A = _dense(m, n, 1)
        Ag = _t(A)
    else:
        A = _csr(m, n, 5, 2)
        Ag = _gpu_csr(A)
    with lib.Context(Ag, mu=1e-4, block=block, seed=seed, max_outer=1, xi=xi) as ctx:
        sz = ctx.sizes()
        s = sz["s"]
        assert s == min(m, math.ceil(1.1 * block))
        rows, signs, xi = orng.sparse_sign(seed, s, m, xi)
        assert sz["xi"] == xi
        np.testing.assert_array_equal(ctx.query(2).reshape(m, xi), rows)       # bit-exact
        np.testing.assert_array_equal(ctx.query(3).reshape(m, xi), signs)
        Y = ctx.query(1).reshape(s, n)
        Yref = orng.sparse_sign_matrix(seed, s, m, xi) @ (A.toarray() if sp.issparse(A) else A)
        assert np.abs(Y - Yref).max() <= 1e-13 * np.abs(Yref).max()
        W = ctx.query(4).reshape(10, n).T
        np.testing.assert_allclose(W, orng.gaussian_probes(seed, n, 10), rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("kind", ["dense", "csr"])
@pytest.mark.parametrize("xi", [1, 3])
def test_sketch_other_xi_matches_oracle(lib, kind, xi):
    test_sketch_matches_oracle(lib, kind, 3001, 120, 20, xi)


@pytest.mark.parametrize("kind,dtype,variant", [("dense", torch.float64, 1), ("dense", torch.float32, 1),
                                                ("dense", torch.float32, 2), ("csr", torch.float64, 1),
                                                ("csr", torch.float32, 1)])
def test_gaussian_sketch_matches_oracle(lib, kind, dtype, variant):
    """Gaussian sketch (option sketch = 1, 2): Y = S A against the oracle's S
    (same counter-based stream) times A.  FP64 products, and CSR with FP64
    accumulation: within 1e-12 of |S| |A| per entry (the Box-Muller values
    agree to a few ulps).  Dense FP32 A, sketch 1: S rounded to FP32 (2^-24
    relative), FP32 MFMA sums of 16 terms (16 2^-24), FP64 across the sums:
    bound 20 2^-24 |S| |A|.  Sketch 2: S and A rounded to BF16 (2^-9 each),
    exact products, 32-term FP32 sums: bound (2^-8 + 2^-17 + 40 2^-24)
    |S| |A|."""
    seed, block, m, n = 13, 20, 3001, 150
    if kind == "dense":
        A = _dense(m, n, 5)
        if dtype == torch.float32:
            A = A.astype(np.float32).astype(np.float64)
        Ag, Ad = _t(A, dtype), A
    else:
        A = _csr(m, n, 5, 6)
        if dtype == torch.float32:
            A = sp.csr_matrix((A.data.astype(np.float32).astype(np.float64), A.indices, A.indptr), shape=A.shape)
        Ag, Ad = _gpu_csr(A, dtype), A.toarray()
    with lib.Context(Ag, mu=1e-4, block=block, seed=seed, max_outer=1, sketch=variant) as ctx:
        s = ctx.sizes()["s"]
        Y = ctx.query(1).reshape(s, n)
        assert ctx.query(2).size == 0
        W = ctx.query(4).reshape(10, n).T
    S = orng.gaussian_sketch(seed, s, m)
    Yref = S @ Ad
    mag = np.abs(S) @ np.abs(Ad)
    tol = 1e-12
    if kind == "dense" and dtype == torch.float32:
        tol = 20 * 2.0 ** -24 if variant == 1 else 2.0 ** -8 + 2.0 ** -17 + 40 * 2.0 ** -24
    err = float(np.max(np.abs(Y - Yref) / (mag + 1e-300)))
    print(f"[parity] Gaussian sketch {kind} {dtype} variant {variant}: max error / (|S||A|) = {err:.3e} "
          f"(bound {tol:.3e})")
    assert np.all(np.abs(Y - Yref) <= tol * mag + 1e-300)
    np.testing.assert_allclose(W, orng.gaussian_probes(seed, n, 10), rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("kind", ["dense", "csr"])
def test_gaussian_sketch_solution_matches_oracle(lib, kind):
    """APLICUR with the Gaussian sketch: the oracle's CUR indices over the
    first outer steps, and the dense-QR solution."""
    if kind == "dense":
        A = _dense(600, 70, 22, decades=5)
        Ag = _t(A)
    else:
        A = _csr(5000, 300, 8, 23, decades=4)
        Ag = _gpu_csr(A)
    b = np.random.default_rng(4).standard_normal(A.shape[0])
    mu, block = 1e-6, 7
    tr = Trace()
    aplicur(A, b, mu, Options(block=block, tol_ne=1e-30, max_rank=3 * block, sketch="gaussian"), tr)
    with lib.Context(Ag, mu=mu, block=block, tol_ne=1e-30, max_rank=3 * block, max_outer=3,
                     sketch="gaussian") as ctx:
        ctx.solve(_t(b))
        J, I = ctx.query(5), ctx.query(6)
    np.testing.assert_array_equal(J, tr.J[:len(J)])
    np.testing.assert_array_equal(I, tr.I[:len(I)])
    x, info = lib.lstsq(Ag, _t(b), mu=mu, block=block, tol_ne=1e-10, sketch="gaussian")
    xr = solve_dense_qr(A, b, mu)
    assert info.status == 0
    check_solution(x.cpu().numpy(), xr, A, b, mu, f"gaussian sketch {kind}")


@pytest.mark.parametrize("kind", ["dense", "csr"])
@pytest.mark.parametrize("schedule", [1, 2])
def test_single_shot_schedules_match_oracle(lib, kind, schedule):
    """Single-shot schedules (Sec. 7.1): the oracle's rank sequence, rebuild
    flags (one build, at the end) and CUR indices; the dense-QR solution."""
    if kind == "dense":
        A = _dense(500, 60, 24, decades=6)
        Ag = _t(A)
    else:
        A = _csr(4000, 250, 8, 25, decades=5)
        Ag = _gpu_csr(A)
    b = np.random.default_rng(5).standard_normal(A.shape[0])
    mu, block, cap, tol = 1e-8, 5, 30, 1e-10
    tr = Trace()
    x_or = aplicur(A, b, mu, Options(block=block, tol_ne=tol, max_rank=cap, schedule=schedule), tr)
    with lib.Context(Ag, mu=mu, block=block, tol_ne=tol, max_rank=cap, schedule=schedule) as ctx:
        x, info = ctx.solve(_t(b))
        ranks, reb = ctx.query(8), ctx.query(9)
        J, I = ctx.query(5), ctx.query(6)
    assert list(ranks) == tr.ranks
    assert list(reb) == [int(v) for v in tr.rebuild]
    assert int(np.sum(reb)) == 1 and info.rebuilds == 1
    np.testing.assert_array_equal(J, tr.J)
    np.testing.assert_array_equal(I, tr.I)
    xr = solve_dense_qr(A, b, mu)
    assert info.status == 0
    check_solution(x.cpu().numpy(), xr, A, b, mu, f"schedule {schedule} {kind} (GPU)")
    check_solution(x_or, xr, A, b, mu, f"schedule {schedule} {kind} (oracle)")


def test_dependent_columns_end_rank_growth(lib):
    """A CUR step whose columns are numerically dependent on C (the block
    Cholesky of C^T C breaks down) is undone and ends the rank growth, as in
    the oracle; the solve reaches its tolerance."""
    r = np.random.default_rng(0)
    A = synth.dense_svd(r, 1200, 1000, synth.paper_sigma(1000, "smooth"))
    b = A @ r.standard_normal(1000)
    tr = Trace()
    aplicur(A, b, 0.0, Options(block=20, tol_ne=1e-8, max_iter=20000), tr)
    with lib.Context(_t(A), mu=0.0, block=20, tol_ne=1e-8, max_iter=20000) as ctx:
        x, info = ctx.solve(_t(b))
        ranks = ctx.query(8)
    assert ranks[-1] == ranks[-2] and abs(int(ranks[-1]) - tr.ranks[-1]) <= 20
    assert info.status == 0 and ne_residual(A, b, x.cpu().numpy(), 0.0) <= 1.5e-8


def test_sketched_cholqr_option_continues_rank_growth(lib):
    """With tc_sketched, a breakdown of chol(C^T C) takes T_C from sketched
    Cholesky QR (the same Gaussian embedding, seed and passes as the oracle's
    tc = "sketched") instead of undoing the step.  Single-shot schedule 2
    grows the CUR to the rank cap before the one build, so the rank sequence
    is decided by the breakdowns alone: by default the growth ends at the
    first breakdown (the rank repeats; 260 in the oracle, where C^T C loses
    positive definiteness at about 1/u, so rounding may move it by a step),
    with the option it reaches the cap of 400 as in the oracle.  The column
    indices equal the oracle's over the first steps; deeper in this
    root-exponential decay the pivot search meets near-ties that the
    summation order of the GPU's products may resolve either way, so only
    the first 100 are required to match (the first mismatch is printed)."""
    r = np.random.default_rng(0)
    A = synth.dense_svd(r, 1200, 1000, synth.paper_sigma(1000, "smooth"))
    b = A @ r.standard_normal(1000)
    mu, opts = 1e-10, dict(block=20, tol_ne=1e-8, max_iter=20000, schedule=2, max_rank=400)
    tr = Trace()
    aplicur(A, b, mu, Options(tc="sketched", **opts), tr)
    out = {}
    for sk in (False, True):
        with lib.Context(_t(A), mu=mu, tc_sketched=sk, **opts) as ctx:
            x, info = ctx.solve(_t(b))
            out[sk] = ([int(v) for v in ctx.query(8)], ctx.query(5), info, x.cpu().numpy())
    (r0, _, i0, x0), (r1, J1, i1, x1) = out[False], out[True]
    print(f"[parity] sketched T_C: GPU ranks {r1} ({i1.iters} it), default {r0} ({i0.iters} it), "
          f"oracle {tr.ranks} ({tr.iters} it)")
    diff = np.flatnonzero(np.asarray(J1) != np.asarray(tr.J))
    print(f"[parity] sketched T_C: first column index differing from the oracle's: "
          f"{int(diff[0]) if diff.size else 'none'} of {len(tr.J)}")
    assert r0[-1] == r0[-2] and 240 <= r0[-1] < 400
    assert r1 == tr.ranks == list(range(20, 401, 20))
    np.testing.assert_array_equal(J1[:100], tr.J[:100])
    assert i0.status == 0 and ne_residual(A, b, x0, mu) <= 1.5e-8
    assert i1.status == 0 and ne_residual(A, b, x1, mu) <= 1.5e-8


def test_solution_with_xi_matches_oracle(lib):
    """A whole APLICUR solve with xi = 4: the same CUR indices as the oracle's
    first outer steps and the dense-QR solution."""
    A = _dense(600, 70, 21, decades=5)
    b = np.random.default_rng(3).standard_normal(600)
    mu, block = 1e-6, 7
    tr = Trace()
    aplicur(A, b, mu, Options(block=block, tol_ne=1e-30, max_rank=3 * block, xi=4), tr)
    with lib.Context(_t(A), mu=mu, block=block, tol_ne=1e-30, max_rank=3 * block, max_outer=3, xi=4) as ctx:
        ctx.solve(_t(b))
        np.testing.assert_array_equal(ctx.query(5), tr.J[:len(ctx.query(5))])
        np.testing.assert_array_equal(ctx.query(6), tr.I[:len(ctx.query(6))])
    x, info = lib.lstsq(_t(A), _t(b), mu=mu, block=block, tol_ne=1e-10, xi=4)
    xr = solve_dense_qr(A, b, mu)
    assert info.status == 0
    check_solution(x.cpu().numpy(), xr, A, b, mu, "xi = 4")


# ----------------------------------------------------------------- products
@pytest.mark.parametrize("kind,dtype", [("dense", torch.float64), ("dense", torch.float32),
                                        ("csr", torch.float64), ("csr", torch.float32)])
@pytest.mark.parametrize("m,n", [(1, 1), (77, 5), (4099, 257), (20000, 700)])
def test_matvec_matches_numpy(lib, kind, dtype, m, n):
    r = np.random.default_rng(m + n)
    if kind == "dense":
        A = r.standard_normal((m, n))
        A = A.astype(np.float32).astype(np.float64) if dtype == torch.float32 else A
        Ag = _t(A, dtype)
        An = A
    else:
        A = _csr(m, n, min(7, n), 3)
        if dtype == torch.float32:
            A.data = A.data.astype(np.float32).astype(np.float64)
        Ag = _gpu_csr(A, dtype)
        An = A
    x = r.standard_normal(n)
    u = r.standard_normal(m)
    with lib.Context(Ag, mu=0.0 if m >= n else 1e-3, precond=False) as ctx:
        y = ctx.matvec(_t(x)).cpu().numpy()
        z = ctx.matvec(_t(u), trans=True).cpu().numpy()
    yr = An @ x
    zr = An.T @ u
    assert np.abs(y - yr).max() <= 1e-12 * (np.abs(An).max() * np.abs(x).sum() + 1e-300)
    assert np.abs(z - zr).max() <= 1e-12 * (np.abs(An).max() * np.abs(u).sum() + 1e-300)


# ----------------------------------------------------------------- plain LSQR
@pytest.mark.parametrize("kind", ["dense", "csr"])
@pytest.mark.parametrize("mu", [0.0, 1e-3])
def test_plain_lsqr_iterates_match_oracle(lib, kind, mu):
    # the first k iterations of the Golub-Kahan/LSQR recurrence, element by
    # element, on well-conditioned inputs (kappa <= 10): there the Lanczos
    # vectors stay orthogonal and the iterates are reproducible to rounding;
    # past the loss of orthogonality two FP64 summation orders legitimately
    # follow different (equally convergent) trajectories.
    if kind == "dense":
        A = _dense(600, 70, 4, decades=1.0)
        Ag = _t(A)
    else:
        A = _csr(3000, 400, 6, 5, decades=0.5)
        Ag = _gpu_csr(A)
    b = np.random.default_rng(9).standard_normal(A.shape[0])
    for k in (1, 2, 7, 25):
        x_ref, it, _ = plsqr_phase(A, math.sqrt(mu), b, np.zeros(A.shape[1]), None, eps_lsqr=0.0,
                                   tol_ne=0.0, max_iter=k)
        with lib.Context(Ag, mu=mu, precond=False, max_iter=k, tol_ne=1e-300) as ctx:
            x, info = ctx.solve(_t(b))
        x = x.cpu().numpy()
        assert info.iters == k
        assert np.linalg.norm(x - x_ref) <= 1e-10 * np.linalg.norm(x_ref)


@pytest.mark.parametrize("kind", ["dense", "csr"])
def test_plain_lsqr_converges_to_oracle_solution(lib, kind):
    mu = 1e-4
    if kind == "dense":
        A = _dense(800, 120, 6, decades=4)
        Ag = _t(A)
    else:
        A = _csr(5000, 500, 8, 7, decades=3)
        Ag = _gpu_csr(A)
    b = np.random.default_rng(10).standard_normal(A.shape[0])
    x, info = lib.lstsq(Ag, _t(b), mu=mu, precond=False, tol_ne=1e-10)
    x = x.cpu().numpy()
    eta = ne_residual(A, b, x, mu)
    assert info.status == 0 and eta <= 1.5e-10 and info.eta <= 1e-10
    xr = solve_dense_qr(A, b, mu)
    check_solution(x, xr, A, b, mu, f"plain LSQR {kind}")
    # iteration counts agree up to the finite-precision trajectory spread
    x_or, it_or = lsqr_plain(A, b, mu, tol_ne=1e-10)
    assert 0.8 * it_or <= info.iters <= 1.25 * it_or


# ----------------------------------------------------------------- APLICUR steps
@pytest.mark.parametrize("kind", ["dense", "csr"])
def test_first_outer_step_indices_and_rho(lib, kind):
    if kind == "dense":
        A = _dense(500, 80, 12, decades=5)
        Ag = _t(A)
    else:
        A = _csr(4000, 300, 6, 13, decades=4)
        Ag = _gpu_csr(A)
    block, seed, mu = 8, 21, 1e-6
    with lib.Context(Ag, mu=mu, block=block, seed=seed, max_outer=1) as ctx:
        ctx.solve(_t(np.ones(A.shape[0])))
        I, J = ctx.query(6), ctx.query(5)
        rho = ctx.query(7)
    s = math.ceil(1.1 * block)
    Y = orng.sparse_sign_matrix(seed, s, A.shape[0]) @ (A.toarray() if sp.issparse(A) else A)
    Ir, Jr, _ = augment_cur(A, Y, np.zeros(0, int), np.zeros(0, int), None, None, None, block)
    np.testing.assert_array_equal(J, Jr)
    np.testing.assert_array_equal(I, Ir)
    _, _, _, E_row = core_and_residual(A, Y, Ir, Jr)
    rho_ref = rho_estimate(E_row, orng.gaussian_probes(seed, A.shape[1], 10))
    assert abs(rho[0] - rho_ref) <= 1e-9 * rho_ref


@pytest.mark.parametrize("kind", ["dense", "csr"])
def test_outer_steps_match_oracle_trace(lib, kind):
    if kind == "dense":
        A = _dense(400, 60, 14, decades=6)
        Ag = _t(A)
    else:
        A = _csr(3000, 200, 6, 15, decades=5)
        Ag = _gpu_csr(A)
    block, seed, mu, steps = 5, 3, 1e-5, 4
    b = np.random.default_rng(1).standard_normal(A.shape[0])
    tr = Trace()
    # the oracle trace of the first `steps` outer steps
    aplicur(A, b, mu, Options(block=block, seed=seed, tol_ne=1e-30, max_rank=block * steps), tr)
    with lib.Context(Ag, mu=mu, block=block, seed=seed, max_outer=steps, tol_ne=1e-30,
                     max_rank=block * steps) as ctx:
        ctx.solve(_t(b))
        ranks, rhos, reb = ctx.query(8), ctx.query(7), ctx.query(9)
        I, J = ctx.query(6), ctx.query(5)
        sig = ctx.query(11)
    n_or = len(tr.ranks)
    assert list(ranks[:n_or]) == tr.ranks[:len(ranks)]
    np.testing.assert_allclose(rhos[:n_or], tr.rhos[:len(rhos)], rtol=1e-7)
    assert list(reb[:n_or]) == [int(v) for v in tr.rebuild[:len(reb)]]
    np.testing.assert_array_equal(J, tr.J[:len(J)])
    np.testing.assert_array_equal(I, tr.I[:len(I)])
    assert len(sig) == ranks[-1]


@pytest.mark.parametrize("kind", ["dense", "csr"])
@pytest.mark.parametrize("mu", [1e-6, 1e-3])
def test_aplicur_solution_matches_oracle(lib, kind, mu):
    if kind == "dense":
        A = _dense(700, 90, 16, decades=6)
        Ag = _t(A)
    else:
        A = _csr(6000, 400, 8, 17, decades=4)
        Ag = _gpu_csr(A)
    b = np.random.default_rng(2).standard_normal(A.shape[0])
    block, tol = 10, 1e-10
    x, info = lib.lstsq(Ag, _t(b), mu=mu, block=block, tol_ne=tol)
    x = x.cpu().numpy()
    eta = ne_residual(A, b, x, mu)
    assert info.status == 0 and eta <= 1.5 * tol
    x_or = aplicur(A, b, mu, Options(block=block, tol_ne=tol))
    xr = solve_dense_qr(A, b, mu)
    check_solution(x, xr, A, b, mu, f"APLICUR {kind} mu={mu} (GPU)")
    check_solution(x_or, xr, A, b, mu, f"APLICUR {kind} mu={mu} (oracle)")


def test_aplicur_workload1_reduced(lib):
    w = synth.workload(1, 0.5)  # 1000 x 100, mu = 0, kappa = 1e6
    x, info = lib.lstsq(_t(w.A), _t(w.B), mu=0.0, block=w.block, tol_ne=w.tol)
    x = x.cpu().numpy()
    eta = ne_residual(w.A, w.B, x, 0.0)
    assert eta <= 1.5 * w.tol
    tr = Trace()
    aplicur(w.A, w.B, 0.0, Options(block=w.block, tol_ne=w.tol), tr)
    assert info.rank == tr.ranks[-1]


def test_zero_rhs_and_warm_start(lib):
    A = _dense(200, 30, 19)
    Ag = _t(A)
    x, info = lib.lstsq(Ag, _t(np.zeros(200)), mu=1e-3, block=4)
    assert float(x.abs().max()) == 0.0 and info.eta == 0.0
    b = np.random.default_rng(5).standard_normal(200)
    xr = solve_dense_qr(A, b, 1e-3)
    with lib.Context(Ag, mu=1e-3, block=4, tol_ne=1e-12) as ctx:
        x0 = _t(xr)
        x1, info = ctx.solve(_t(b), X0=x0)
        assert info.iters <= 5
        assert np.linalg.norm(x1.cpu().numpy() - xr) <= 1e-9 * np.linalg.norm(xr)


# ----------------------------------------------------------------- full size (the benchmark workload)
@pytest.fixture(scope="module")
def workload2():
    return synth.workload(2, 1.0)  # CSR 200000 x 20000, 2.0e6 non-zeros, mu = 1e-4


def test_full_size_products(lib, workload2):
    A = workload2.A
    m, n = A.shape
    r = np.random.default_rng(21)
    x, u = r.standard_normal(n), r.standard_normal(m)
    with lib.Context(_gpu_csr(A), mu=workload2.mu, precond=False) as ctx:
        y = ctx.matvec(_t(x)).cpu().numpy()
        z = ctx.matvec(_t(u), trans=True).cpu().numpy()
    yr, zr = A @ x, A.T @ u
    assert np.abs(y - yr).max() <= 1e-13 * (abs(A).max() * np.abs(x).max() * 10)
    assert np.abs(z - zr).max() <= 1e-13 * (abs(A).max() * np.abs(u).max() * abs(A).getnnz(axis=0).max())


def _lds_case(shape):
    r = np.random.default_rng(33)
    m, n = 150037, 16000  # m not a multiple of the 64-row slices
    lens = r.integers(8, 14, m)
    if shape == "skewed_rows":
        lens[r.choice(m, 200, replace=False)] = 3000  # padding the slices would cost far more than a quarter
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    ci = r.integers(0, n, int(rp[-1]))
    val = r.standard_normal(int(rp[-1])) * np.exp(r.uniform(-3, 3, int(rp[-1])))
    return sp.csr_matrix((val, ci, rp), shape=(m, n))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("shape", ["uniform_rows", "skewed_rows"])
def test_lds_resident_products(lib, shape, dtype):
    """A x with x held in LDS (at least 1.5e6 non-zeros, n small enough):
    through the SELL-64 copy when rows are near-uniform, through the CSR row
    blocks when a few long rows would make the padding too large."""
    A = _lds_case(shape)
    if dtype == torch.float32:
        A = sp.csr_matrix((A.data.astype(np.float32).astype(np.float64), A.indices, A.indptr), shape=A.shape)
    m, n = A.shape
    r = np.random.default_rng(22)
    x, u = r.standard_normal(n), r.standard_normal(m)
    with lib.Context(_gpu_csr(A, dtype), mu=1e-4, precond=False) as ctx:
        y = ctx.matvec(_t(x)).cpu().numpy()
        z = ctx.matvec(_t(u), trans=True).cpu().numpy()
        # x not 16-byte aligned (a view one entry into a buffer): the copy of x
        # into LDS takes its single-entry path; the sums are the same
        xb = torch.zeros(n + 1, dtype=torch.float64, device=DEV)
        xb[1:] = _t(x)
        assert xb[1:].data_ptr() % 16 == 8
        y_un = ctx.matvec(xb[1:]).cpu().numpy()
    np.testing.assert_array_equal(y_un, y)
    yr, zr = A @ x, A.T @ u
    absA = abs(A)
    assert np.abs(y - yr).max() <= 1e-13 * (absA @ np.abs(x)).max()
    assert np.abs(z - zr).max() <= 1e-13 * (absA.T @ np.abs(u)).max()


def _uniform_csr(m, n, per_row, seed):
    """per_row distinct columns in every row (a random start, then steps of n / per_row)."""
    r = np.random.default_rng(seed)
    ci = (r.integers(0, n, (m, 1)) + (n // per_row) * np.arange(per_row)[None, :]) % n
    ci = np.sort(ci, axis=1).reshape(-1)
    rp = np.arange(0, m * per_row + 1, per_row)
    return sp.csr_matrix((r.standard_normal(m * per_row), ci, rp), shape=(m, n))


@pytest.mark.parametrize("n", [20352, 20353])
def test_lds_products_at_the_size_limit(lib, n):
    """x in LDS holds at most 159 KB: n = 20352 FP64 entries is the largest n
    the LDS-resident product takes (the whole copy in one batch), n + 1 takes
    the other path; both give A x within the FP64 bound."""
    A = _uniform_csr(150016, n, 10, n)
    x = np.random.default_rng(1).standard_normal(n)
    with lib.Context(_gpu_csr(A), mu=1e-4, precond=False) as ctx:
        y = ctx.matvec(_t(x)).cpu().numpy()
    assert np.abs(y - A @ x).max() <= 1e-13 * (abs(A) @ np.abs(x)).max()


def test_fp32_phases_at_the_lds_size_limit(lib):
    """FP32 phases keep x in LDS up to n = 40704 FP32 entries (159 KB); the
    solve reaches the FP64 tolerance through that largest copy."""
    n = 40704
    A = _uniform_csr(160000, n, 10, 5)
    b = np.random.default_rng(6).standard_normal(A.shape[0])
    x, info = lib.lstsq(_gpu_csr(A), _t(b), mu=1e-1, precond=False, precision=1, tol_ne=1e-8)
    assert info.status == 0
    assert ne_residual(A, b, x.cpu().numpy(), 1e-1) <= 1.05e-8


def test_full_size_fp32_phases(lib, workload2):
    """FP32 LSQR phases (FP32 values, A x from the FP32 SELL copy) with FP64
    refinement reach the FP64 tolerance at the benchmark size."""
    w = workload2
    x, info = lib.lstsq(_gpu_csr(w.A), _t(w.B), mu=w.mu, block=w.block, tol_ne=w.tol, precond=True,
                        max_rank=256, precision=1)
    eta = ne_residual(w.A, w.B, x.cpu().numpy(), w.mu)
    assert info.status == 0
    assert eta <= 1.05 * w.tol
    assert abs(eta - info.eta) <= 1e-3 * w.tol


@pytest.mark.parametrize("precond", [False, True])
def test_full_size_solve_reaches_tolerance(lib, workload2, precond):
    """At the benchmark size the solution is checked through the normal-equation
    residual recomputed on the CPU in FP64 (the oracle's metric)."""
    w = workload2
    x, info = lib.lstsq(_gpu_csr(w.A), _t(w.B), mu=w.mu, block=w.block, tol_ne=w.tol, precond=precond,
                        max_rank=512)
    eta = ne_residual(w.A, w.B, x.cpu().numpy(), w.mu)
    assert info.status == 0
    assert eta <= 1.05 * w.tol
    assert abs(eta - info.eta) <= 1e-3 * w.tol


def test_rank_cap_matches_oracle(lib):
    """The rank cap cuts the last increment on both sides (ranks 10, 20, 25)."""
    A = synth.dense_svd(np.random.default_rng(9), 300, 80, 10.0 ** (-8 * np.arange(80) / 79))
    b = np.random.default_rng(10).standard_normal(300)
    tr = Trace()
    x_or = aplicur(A, b, 1e-12, Options(block=10, tol_ne=1e-10, max_rank=25), tr)
    with lib.Context(_t(A), mu=1e-12, block=10, tol_ne=1e-10, max_rank=25) as ctx:
        x, info = ctx.solve(_t(b))
        ranks = ctx.query(8).tolist()
        np.testing.assert_array_equal(np.sort(ctx.query(5)), np.sort(tr.J))
        np.testing.assert_array_equal(np.sort(ctx.query(6)), np.sort(tr.I))
    assert ranks == tr.ranks == [10, 20, 25]
    assert info.eta <= 1.5e-10
    xr = solve_dense_qr(A, b, 1e-12)
    check_solution(x.cpu().numpy(), xr, A, b, 1e-12, "rank cap (GPU)")
    check_solution(x_or, xr, A, b, 1e-12, "rank cap (oracle)")


def test_product_timer_warm_and_cold(lib):
    """aplicur_time_product: finite positive durations with warm caches and
    with a flush buffer read and written before each timed launch; the flush
    leaves the product's result unchanged (y is recomputed each round) and
    bad flush sizes are rejected."""
    A = _csr(20000, 2000, 8, 31, decades=2)
    x = np.random.default_rng(31).standard_normal(2000)
    flush = torch.zeros(1 << 24, dtype=torch.int32, device=DEV)  # 64 MiB
    with lib.Context(_gpu_csr(A), mu=1e-4, precond=False) as ctx:
        xv = _t(x)
        warm = ctx.time_product(xv, reps=5)
        cold = ctx.time_product(xv, reps=5, flush=flush)
        cold_t = ctx.time_product(xv, trans=True, reps=5, flush=flush)
        assert all(np.isfinite(v) and v > 0 for v in (warm, cold, cold_t))
        assert int(flush[0]) == 10 and int(flush[-1]) == 10  # one pass per round
        with pytest.raises(RuntimeError, match="flush_bytes"):
            ctx.time_product(xv, reps=1, flush=flush[:3])
        y = ctx.matvec(xv).cpu().numpy()
    assert np.abs(y - A @ x).max() <= 1e-13 * (abs(A) @ np.abs(x)).max()
