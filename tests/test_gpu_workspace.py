"""Caller workspace (aplicur_workspace_bytes + aplicur_sketch with ws): every
device buffer of the context is carved from one PyTorch tensor; results equal
the library-allocated context's bit for bit (same kernels, same order)."""
import numpy as np
import pytest
import torch

from workloads import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV, dtype=dtype)


def _dense(m, n, seed, decades=3.0):
    r = np.random.default_rng(seed)
    return synth.dense_svd(r, m, n, 10.0 ** (-decades * np.arange(n) / max(n - 1, 1)))


def _same(lib, A, B, opts, k):
    with lib.Context(A, **opts) as ctx:
        X0, i0 = ctx.solve(B)
    with lib.Context(A, workspace=k, **opts) as ctx:
        assert ctx.workspace is not None and ctx.workspace.numel() > 0
        X1, i1 = ctx.solve(B)
    assert i0.status == i1.status == 0 and i0.iters == i1.iters
    assert torch.equal(X0, X1)


@pytest.mark.parametrize("precision", [0, 1, 2])
@pytest.mark.parametrize("k", [1, 8])
def test_dense_workspace_matches_library_allocation(lib, precision, k):
    A = _t(_dense(700, 90, 81, decades=4))
    B = _t(np.random.default_rng(82).standard_normal((700, k)))
    _same(lib, A, B, dict(mu=1e-5, block=10, tol_ne=1e-10, precision=precision), k)


@pytest.mark.parametrize("precision", [0, 1])
def test_csr_workspace_matches_library_allocation(lib, precision):
    import paper_2604_05065_amd as ap
    A = synth.sparse_scaled(np.random.default_rng(83), 5000, 300, 8, 3.0)
    Ag = ap.CSRMatrix.from_scipy(A, device=DEV, dtype=torch.float64)
    B = _t(np.random.default_rng(84).standard_normal((5000, 2)))
    _same(lib, Ag, B, dict(mu=1e-6, block=10, tol_ne=1e-10, precision=precision), 2)


def test_adjoint_in_workspace(lib):
    A = _t(_dense(600, 70, 85, decades=2))
    r = np.random.default_rng(86)
    B, G = _t(r.standard_normal((600, 4))), _t(r.standard_normal((70, 4)))
    opts = dict(mu=1e-3, block=8, tol_ne=1e-11)
    out = []
    for ws in (0, 4):
        with lib.Context(A, workspace=ws, **opts) as ctx:
            X, _ = ctx.solve(B)
            out.append((X,) + tuple(ctx.solve_backward(X, B, G)[:3]))
    for a, b in zip(*out):
        assert torch.equal(a, b)


def test_workspace_too_small_for_more_columns(lib):
    """Sized for one column, a 16-column blocked solve runs out of it."""
    A = _t(_dense(500, 60, 87))
    B = _t(np.random.default_rng(88).standard_normal((500, 16)))
    with lib.Context(A, workspace=1, mu=1e-4, block=6) as ctx:
        x, info = ctx.solve(B[:, 0])
        assert info.status == 0
        with pytest.raises(RuntimeError, match="workspace"):
            ctx.solve(B)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_column_major_input(lib, dtype):
    """A column-major A (a transposed view, format DENSE_COL) gives the
    row-major input's results: solves bit for bit (the context keeps a
    row-major copy), dA in A's column-major layout."""
    A = _dense(500, 60, 89, decades=2)
    Arow = _t(A, dtype)
    Acol = _t(A.T, dtype).t()  # same values, column-major storage
    assert Acol.stride() == (1, 500)
    r = np.random.default_rng(90)
    B, G = _t(r.standard_normal((500, 3))), _t(r.standard_normal((60, 3)))
    opts = dict(mu=1e-3, block=8, tol_ne=1e-11)
    res = []
    for Am in (Arow, Acol):
        with lib.Context(Am, **opts) as ctx:
            X, info = ctx.solve(B)
            Z, dB, dA, _ = ctx.solve_backward(X, B, G)
        res.append((X, Z, dB, dA))
    for a, b in zip(res[0][:3], res[1][:3]):
        assert torch.equal(a, b)
    assert res[1][3].stride() == (1, 500)
    assert torch.allclose(res[0][3], res[1][3], rtol=1e-12, atol=1e-12 * float(res[0][3].abs().max()))


def test_reused_workspace_tensor(lib):
    """One caller tensor of workspace_bytes(A, k) bytes serves one context
    after another (different sketch seeds), each bitwise equal to the
    library-allocated context of the same seed; a tensor far short of the
    need fails with E_NOMEM instead of writing past it."""
    import paper_2604_05065_amd as ap
    A = _t(_dense(900, 120, 87, decades=4))
    B = _t(np.random.default_rng(88).standard_normal((900, 16)))
    opts = dict(mu=1e-6, block=12, tol_ne=1e-10)
    need = max(ap.workspace_bytes(A, 16, seed=s, **opts) for s in (3, 4))
    ws = torch.empty(need, dtype=torch.uint8, device=DEV)
    for seed in (3, 4, 3):
        with lib.Context(A, seed=seed, **opts) as ctx:
            X0, i0 = ctx.solve(B)
        with lib.Context(A, workspace=ws, seed=seed, **opts) as ctx:
            assert ctx.workspace is ws
            X1, i1 = ctx.solve(B)
        assert i0.status == i1.status == 0 and i0.iters == i1.iters
        assert torch.equal(X0, X1)
    short = torch.empty(1 << 16, dtype=torch.uint8, device=DEV)
    with pytest.raises(ap.AplicurError):
        with lib.Context(A, workspace=short, seed=3, **opts) as ctx:
            ctx.solve(B)
