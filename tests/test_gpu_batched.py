"""Batched solves (worker streams, graph replay, tile autotuning) against
one-at-a-time solves and the oracle -- GPU tests through the C ABI."""
import numpy as np
import pytest
import torch

from oracle.aplicur import ne_residual
from oracle.dense import solve_dense_qr
from workloads import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV, dtype=dtype)


def _batch(count=7, nrhs=2):
    """Uneven dense and CSR problems (sizes like a scaled-down batched workload)."""
    r = np.random.default_rng(70)
    probs = []
    for i in range(count):
        m = int(r.integers(300, 2500))
        n = int(r.integers(20, max(21, min(200, m // 4))))
        if i % 3 == 2:
            A = synth.sparse_scaled(r, m, n, 6, float(r.uniform(1, 4)))
        else:
            A = synth.dense_svd(r, m, n, 10.0 ** (-r.uniform(2, 5) * np.arange(n) / max(n - 1, 1)))
        probs.append((A, r.standard_normal((m, nrhs))))
    return probs


def _gpu(lib, A, dtype=torch.float64):
    if hasattr(A, "tocsr"):
        return lib.CSRMatrix.from_scipy(A, device=DEV, dtype=dtype)
    return _t(A, dtype)


OPTS = dict(mu=1e-6, block=8, tol_ne=1e-10)


@pytest.mark.parametrize("precond", [True, False])
def test_batched_equals_one_at_a_time(lib, precond):
    """Worker streams and graph replay change nothing in the arithmetic: with
    fixed tiles every solution is bitwise the one-at-a-time solution."""
    probs = _batch()
    As = [_gpu(lib, A) for A, _ in probs]
    Bs = [_t(B) for _, B in probs]
    Xs, infos = lib.solve_batched(As, Bs, workers=3, tune=False, graphs=True, precond=precond, **OPTS)
    for (A, B), Ag, Bg, X, info in zip(probs, As, Bs, Xs, infos):
        Xr, ir = lib.lstsq(Ag, Bg, precond=precond, **OPTS)
        assert info.status == 0 and info.iters == ir.iters and info.rank == ir.rank
        assert torch.equal(X, Xr)
        for k in range(B.shape[1]):
            assert ne_residual(A, B[:, k], X[:, k].cpu().numpy(), OPTS["mu"]) <= 1.5 * OPTS["tol_ne"]


def test_batched_many_workers_capture_while_others_set_up(lib):
    """Eight workers: graph captures overlap other workers' context set-up,
    library calls and releases (guarded by the library)."""
    probs = _batch(count=12, nrhs=1)
    As = [_gpu(lib, A) for A, _ in probs]
    Bs = [_t(B[:, 0]) for _, B in probs]
    for tune in (True, False):
        Xs, infos = lib.solve_batched(As, Bs, workers=8, tune=tune, graphs=True, **OPTS)
        for (A, B), X, info in zip(probs, Xs, infos):
            assert info.status == 0
            assert ne_residual(A, B[:, 0], X.cpu().numpy(), OPTS["mu"]) <= 1.5 * OPTS["tol_ne"]


def test_batched_tuned_tiles(lib):
    """With autotuned tiles the summation order may differ; the solutions
    still meet the tolerance and agree with dense QR."""
    probs = _batch(count=5, nrhs=1)
    As = [_gpu(lib, A) for A, _ in probs]
    Bs = [_t(B[:, 0]) for _, B in probs]
    Xs, infos = lib.solve_batched(As, Bs, workers=4, tune=True, graphs=True, **OPTS)
    for (A, B), X, info in zip(probs, Xs, infos):
        x = X.cpu().numpy()
        assert info.status == 0
        assert ne_residual(A, B[:, 0], x, OPTS["mu"]) <= 1.5 * OPTS["tol_ne"]
        xr = solve_dense_qr(A, B[:, 0], OPTS["mu"])
        assert np.linalg.norm(x - xr) <= 1e-5 * np.linalg.norm(xr)


@pytest.mark.parametrize("kind", ["dense", "csr"])
def test_graph_replay_matches_eager(lib, kind):
    """Captured LSQR chunks replayed many times (with the host's own state
    reads and refinement work between replays) give the eager result bit for bit."""
    r = np.random.default_rng(71)
    if kind == "dense":
        A = synth.dense_svd(r, 1500, 120, 10.0 ** (-4 * np.arange(120) / 119))
    else:
        A = synth.sparse_scaled(r, 6000, 300, 8, 3.0)
    b = r.standard_normal(A.shape[0])
    Ag, bg = _gpu(lib, A), _t(b)
    side = torch.cuda.Stream()
    for precond in (False, True):
        x0, i0 = lib.lstsq(Ag, bg, graphs=False, precond=precond, **OPTS)
        with torch.cuda.stream(side):
            x1, i1 = lib.lstsq(Ag, bg, graphs=True, precond=precond, **OPTS)
            x2, i2 = lib.lstsq(Ag, bg, graphs=True, precond=precond, precision=1, **OPTS)
        torch.cuda.synchronize()
        assert i1.iters == i0.iters
        if not precond:
            assert i1.iters > 3 * 16  # several replays of the 16-iteration graph
        assert torch.equal(x0, x1)
        assert i2.status == 0 and ne_residual(A, b, x2.cpu().numpy(), OPTS["mu"]) <= 1.5 * OPTS["tol_ne"]


def test_batched_rejects_invalid_problem(lib):
    r = np.random.default_rng(72)
    As = [_t(r.standard_normal((50, 10))), _t(r.standard_normal((5, 10)))]  # second: m < n with mu = 0
    Bs = [_t(r.standard_normal(50)), _t(r.standard_normal(5))]
    with pytest.raises(lib.AplicurError):
        lib.solve_batched(As, Bs, mu=0.0)


def test_batched_caller_workspace(lib):
    """With a caller workspace (aplicur_batched_workspace_bytes, one slice
    per worker) every context is carved from it, and the solutions are
    bitwise those of the library-allocated run; one byte short is rejected
    with the size in the message before any problem runs."""
    probs = _batch(count=6)
    As = [_gpu(lib, A) for A, _ in probs]
    Bs = [_t(B) for _, B in probs]
    kw = dict(workers=3, tune=False, graphs=True, **OPTS)
    need = lib.batched_workspace_bytes(As, 2, **kw)
    assert need > 0
    ws = torch.empty(need, dtype=torch.uint8, device=DEV)
    assert ws.data_ptr() % 256 == 0
    Xw, iw = lib.solve_batched(As, Bs, workspace=ws, **kw)
    Xr, ir = lib.solve_batched(As, Bs, **kw)
    print(f"[batched] workspace {need} bytes for 3 workers")
    for a, b, ia, ib in zip(Xw, Xr, iw, ir):
        assert ia.status == 0 and ia.iters == ib.iters
        assert torch.equal(a, b)
    with pytest.raises(lib.AplicurError, match="workspace needs"):
        lib.solve_batched(As, Bs, workspace=ws[: need - 256], **kw)
