"""aplicur_sketch_noalloc (no device allocation; scratch in a fixed
per-device array) against the sketch of aplicur_sketch (Alg. 3
initialisation, Definition 5.1) on the same inputs: two calls in a row, the
second with a smaller input, for dense and CSR A.  Both run the same kernels
in the same summation order, so the two must agree bit for bit; both are also
held to the FP64 sketch bound against the oracle's S A (every entry a sum of
at most m terms |S_hi a_ij|, 1e-13 of their magnitudes)."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

from oracle import rng as orng
from workloads import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _case(kind, m, n, seed, dtype):
    r = np.random.default_rng(seed)
    if kind == "dense":
        A = synth.dense_svd(r, m, n, 10.0 ** (-3 * np.arange(n) / max(n - 1, 1)))
        if dtype == torch.float32:
            A = A.astype(np.float32).astype(np.float64)
        return A, torch.as_tensor(A, device=DEV, dtype=dtype)
    A = synth.sparse_scaled(r, m, n, 9, 2.0)
    if dtype == torch.float32:
        A.data = A.data.astype(np.float32).astype(np.float64)
    import paper_2604_05065_amd as ap
    return A, ap.CSRMatrix.from_scipy(A, device=DEV, dtype=dtype)


@pytest.mark.parametrize("kind", ["dense", "csr"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_sketch_noalloc_matches_sketch(lib, kind, dtype):
    sizes = [(6000, 500, 100), (1100, 90, 20)] if kind == "dense" else [(40000, 3000, 100), (3000, 200, 20)]
    for call, (m, n, block) in enumerate(sizes):
        seed = 31 + call
        A, Ag = _case(kind, m, n, 5 + call, dtype)
        print(f"[no-alloc] {kind} {dtype} call {call}: {m} x {n}, block {block}", flush=True)
        Y = lib.sketch_noalloc(Ag, block=block, seed=seed)
        torch.cuda.synchronize()
        with lib.Context(Ag, mu=1e-4, block=block, seed=seed, max_outer=1) as ctx:
            s = ctx.sizes()["s"]
            Yref = ctx.query(1).reshape(s, n)
        Yn = Y.cpu().numpy()
        assert Yn.shape == (s, n)
        S = orng.sparse_sign_matrix(seed, s, m, 8)
        Ad = A.toarray() if sp.issparse(A) else A
        mag = np.asarray(abs(S) @ np.abs(Ad))
        print(f"[no-alloc]   bitwise equal to aplicur_sketch: {np.array_equal(Yn, Yref)}; "
              f"max |diff| {np.abs(Yn - Yref).max():.3e}", flush=True)
        np.testing.assert_array_equal(Yn, Yref)
        assert np.all(np.abs(Yn - np.asarray(S @ Ad)) <= 1e-13 * mag + 1e-300)
