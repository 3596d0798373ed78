"""The paper's test families (Sec. 6.3: dense U Sigma V^T, incoherent or
coherent, sharp (kappa 1e7, 1e15) or smooth (kappa 1e15) decay, consistent-x
right-hand sides with noise 0, 1e-12 or 1e-2; sparse 1% density, incoherent
or coherent) at reduced sizes, b = n/50 as in the paper's baseline: the
library's APLICUR against the oracle's on the same matrix and right-hand side.

* Incoherent families: the CUR sequence (ranks, I, J) equals the oracle's
  bit for bit, and rho_k agrees to 1e-9 relative or within 100 u cond(W_k)
  rho_1: rho comes from the sketched residual Y - Y(:, J) U R, formed by
  cancellation; the two sides sum the sketch in different orders, a
  difference of a few u ||Y|| (the scale of the first rho), which the core
  inverse U = W^{-1} amplifies by up to cond(W).  Once the CUR has captured
  the spectrum down to a flat tail, rho sits near that floor and only the
  absolute agreement is meaningful.  Coherent families have rows
  and columns that differ only by 1e-8 J, so near-ties of the pivot search
  may resolve differently under a different summation order of the sketch;
  there the first outer step's indices are compared, and the rest through
  the solution.
* Every family: both solutions within the conditioning bound of
  tests/bounds.py of the dense QR reference, and eta <= tol_ne.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

from oracle.aplicur import Options, Trace, aplicur, ne_residual
from oracle.dense import solve_dense_qr
from workloads import synth

from bounds import check_solution

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

# (kind, m, n, decay, coherent, noise, mu)
FAMILIES = [
    ("dense", 600, 500, "sharp7", False, 1e-2, 1e-4),
    ("dense", 600, 500, "sharp7", False, 0.0, 1e-4),
    ("dense", 600, 500, "sharp7", False, 1e-12, 1e-4),
    ("dense", 600, 500, "sharp15", False, 1e-2, 1e-8),
    ("dense", 600, 500, "sharp15", False, 1e-2, 0.0),
    ("dense", 600, 500, "sharp7", True, 1e-2, 1e-4),
    ("dense", 600, 500, "smooth", False, 1e-2, 1e-6),
    ("dense", 1500, 200, "sharp7", False, 1e-2, 1e-4),
    ("sparse", 1200, 1000, "sharp7", False, None, 1e-4),
    ("sparse", 1200, 1000, "sharp7", True, None, 1e-4),
    ("sparse", 3000, 400, "smooth", True, None, 1e-4),
]


def _ids(f):
    kind, m, n, decay, coh, noise, mu = f
    return f"{kind}-{m}x{n}-{decay}-{'coh' if coh else 'inc'}-noise{noise}-mu{mu}"


def _problem(kind, m, n, decay, coh, noise, seed):
    import paper_2604_05065_amd as ap
    if kind == "dense":
        Ag, bg = synth.paper_dense_gpu(seed, m, n, decay, coherent=coh, noise=noise)
        return Ag.cpu().numpy(), bg.cpu().numpy(), Ag, bg
    A, b = synth.paper_sparse(seed, m, n, decay, coherent=coh)
    return A, b, ap.CSRMatrix.from_scipy(A, device=DEV, dtype=torch.float64), torch.as_tensor(b, device=DEV)


@pytest.mark.parametrize("fam", FAMILIES, ids=_ids)
def test_paper_family_matches_oracle(lib, fam):
    kind, m, n, decay, coh, noise, mu = fam
    A, b, Ag, bg = _problem(kind, m, n, decay, coh, noise, 700 + m + n)
    block, tol = max(1, n // 50), 1e-10
    opts = dict(block=block, tol_ne=tol, max_iter=20000)
    tr = Trace()
    x_or = aplicur(A, b, mu, Options(**opts), tr)
    with lib.Context(Ag, mu=mu, **opts) as ctx:
        x, info = ctx.solve(bg)
        ranks, rhos = list(ctx.query(8)), ctx.query(7)
        I, J = ctx.query(6), ctx.query(5)
    x = x.cpu().numpy()
    print(f"[parity] {_ids(fam)}: GPU ranks {ranks}, oracle ranks {tr.ranks}, iters {info.iters}, "
          f"eta {info.eta:.2e}")
    assert info.status == 0 and ne_residual(A, b, x, mu) <= 1.5 * tol
    if coh:
        assert ranks[0] == tr.ranks[0]
        np.testing.assert_array_equal(J[:ranks[0]], tr.J[:ranks[0]])
        np.testing.assert_array_equal(I[:ranks[0]], tr.I[:ranks[0]])
    else:
        assert ranks == tr.ranks
        np.testing.assert_array_equal(J, tr.J)
        np.testing.assert_array_equal(I, tr.I)
        scale = abs(tr.rhos[0])
        for k, (rg, ro) in enumerate(zip(rhos, tr.rhos)):
            l = tr.ranks[k]
            W = A[tr.I[:l], :][:, tr.J[:l]]
            condW = np.linalg.cond(W.toarray() if sp.issparse(W) else W)
            assert abs(rg - ro) <= 1e-9 * abs(ro) + 100 * 2.0 ** -53 * condW * scale, (k, rg, ro, condW)
    Ad = A.toarray() if sp.issparse(A) else A
    xr = solve_dense_qr(Ad, b, mu)
    check_solution(x, xr, Ad, b, mu, f"{_ids(fam)} (GPU)")
    check_solution(x_or, xr, Ad, b, mu, f"{_ids(fam)} (oracle)")
