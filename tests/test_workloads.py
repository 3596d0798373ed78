"""The paper's test-set generators (inputs only): the prescribed spectra and
the sparse family's column scaling."""
import numpy as np

from workloads import synth


def test_paper_sigma():
    n = 5000
    s7, s15, sm = (synth.paper_sigma(n, d) for d in ("sharp7", "sharp15", "smooth"))
    for s in (s7, s15, sm):
        assert s.shape == (n,) and np.all(np.diff(s) <= 0) and s[0] == 100.0
    assert np.isclose(s7[999], 1e-2) and np.isclose(s7[1000], 10 ** -4.8) and np.isclose(s7[-1], 1e-5)
    assert np.isclose(s15[1000], 1e-12) and np.isclose(s15[-1], 1e-13)
    assert np.isclose(sm[-1], 1e-13) and np.isclose(sm[0] / sm[-1], 1e15)
    # root-exponential: log10 sigma is linear in sqrt(i)
    t = np.sqrt(np.arange(n) / (n - 1))
    np.testing.assert_allclose(np.log10(sm), 2 - 15 * t, atol=1e-12)


def test_paper_sparse_columns():
    for coherent in (False, True):
        A, b = synth.paper_sparse(3, 1500, 400, "sharp7", coherent=coherent)
        assert abs(A.nnz - 0.01 * 1500 * 400) < 6 * np.sqrt(0.01 * 1500 * 400)
        norms = np.sqrt(np.asarray(A.multiply(A).sum(axis=0))).ravel()
        live = norms > 0
        np.testing.assert_allclose(norms[live], synth.paper_sigma(400, "sharp7")[live], rtol=1e-12)
        assert b.shape == (1500,)
