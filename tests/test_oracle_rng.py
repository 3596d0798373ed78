"""Pins of the oracle's random stream (sparse sign embedding, Definition 5.1;
Gaussian probes of the 2-norm bound, Sec. 5.3.1)."""
import math
import os

import numpy as np
import pytest

from oracle import rng


GOLDEN_DIR = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_known_answer():
    # Published SplitMix64 sequence from state 0 (the fixture cites its source)
    with open(os.path.join(GOLDEN_DIR, "splitmix64_state0.txt")) as f:
        expected = [int(line, 16) for line in f if line.strip() and not line.startswith("#")]
    state = np.uint64(0)
    outs = []
    for _ in range(len(expected)):
        with np.errstate(over="ignore"):
            state = state + rng.GOLDEN
        outs.append(int(rng.mix64(state)))
    assert len(expected) == 3 and outs == expected


def test_draw_is_stream_offset():
    # draw(seed, stream, c) is output c of SplitMix64 started at key(seed, stream)
    k = int(rng.key(123, 4))
    with np.errstate(over="ignore"):
        st = np.uint64(k)
        seq = []
        for _ in range(5):
            st = st + rng.GOLDEN
            seq.append(int(rng.mix64(st)))
    assert [int(v) for v in rng.draw(123, 4, np.arange(5))] == seq


@pytest.mark.parametrize("s,m", [(22, 500), (5, 300), (110, 2000), (1, 40), (8, 64)])
def test_sparse_sign_structure(s, m):
    rows, signs, xi = rng.sparse_sign(7, s, m)
    assert xi == min(8, s)
    assert rows.shape == (m, xi) and signs.shape == (m, xi)
    assert rows.min() >= 0 and rows.max() < s
    for i in range(m):
        assert len(set(rows[i].tolist())) == xi  # distinct rows
    assert set(np.unique(signs).tolist()) <= {-1.0, 1.0}
    S = rng.sparse_sign_matrix(7, s, m).toarray()
    # every column of S has unit 2-norm exactly (xi entries of 1/sqrt(xi))
    np.testing.assert_allclose(np.linalg.norm(S, axis=0), 1.0, rtol=0, atol=1e-15)
    assert np.all(np.count_nonzero(S, axis=0) == xi)


@pytest.mark.parametrize("xi", [1, 3, 5, 8])
@pytest.mark.parametrize("s,m", [(22, 500), (4, 300)])
def test_sparse_sign_other_xi(xi, s, m):
    """xi' = min(xi, s) distinct rows per column, entries +-1/sqrt(xi'), unit
    columns; a column's t-th draw does not depend on xi (the counters give
    each column 8 slots), so the xi' rows are the first xi' of the default's
    when xi' <= 8; out-of-range xi is refused."""
    rows, signs, k = rng.sparse_sign(7, s, m, xi)
    assert k == min(xi, s)
    for i in range(m):
        assert len(set(rows[i].tolist())) == k
    S = rng.sparse_sign_matrix(7, s, m, xi).toarray()
    np.testing.assert_allclose(np.linalg.norm(S, axis=0), 1.0, rtol=0, atol=1e-15)
    assert np.all(np.count_nonzero(S, axis=0) == k)
    r8, s8, _ = rng.sparse_sign(7, s, m)
    np.testing.assert_array_equal(rows, r8[:, :k])
    np.testing.assert_array_equal(signs, s8[:, :k])
    for bad in (0, 9):
        with pytest.raises(ValueError):
            rng.sparse_sign(7, s, m, bad)


def test_sparse_sign_statistics():
    s, m = 50, 40000
    rows, signs, xi = rng.sparse_sign(11, s, m)
    # sign balance: binomial(320000, 1/2) -> 6 sigma band
    frac = np.mean(signs > 0)
    assert abs(frac - 0.5) < 6 * 0.5 / math.sqrt(signs.size)
    # rows uniform: chi-square with s - 1 dof far below its 1e-6 tail
    counts = np.bincount(rows.reshape(-1), minlength=s)
    expected = rows.size / s
    chi2 = np.sum((counts - expected) ** 2 / expected)
    assert chi2 < 120.0
    # a different seed gives a different embedding
    rows2, _, _ = rng.sparse_sign(12, s, m)
    assert np.mean(rows2 != rows) > 0.9


def test_sketch_matches_brute_force():
    # Y = S A against an explicitly assembled S and dense product
    r = np.random.default_rng(0)
    A = r.standard_normal((60, 9))
    rows, signs, xi = rng.sparse_sign(3, 13, 60)
    S = np.zeros((13, 60))
    for i in range(60):
        for t in range(xi):
            S[rows[i, t], i] += signs[i, t] / math.sqrt(xi)
    np.testing.assert_allclose(rng.sparse_sign_matrix(3, 13, 60) @ A, S @ A, rtol=1e-14, atol=1e-14)


def test_gaussian_probes():
    W = rng.gaussian_probes(5, 50000, 4)
    assert W.shape == (50000, 4)
    assert abs(W.mean()) < 6 / math.sqrt(W.size)
    assert abs(W.var() - 1.0) < 6 * math.sqrt(2.0 / W.size)
    # Kolmogorov-Smirnov distance to N(0,1) well inside the 1e-6 critical value
    from scipy.stats import kstest
    assert kstest(W[:, 0], "norm").pvalue > 1e-6
    # columns are independent streams
    assert abs(np.corrcoef(W[:, 0], W[:, 1])[0, 1]) < 0.03


def test_gaussian_sketch():
    """Gaussian embedding: N(0, 1/s) entries (mean and variance within 6
    standard errors), E ||S x||^2 = ||x||^2 on average over columns, column
    order independent of m, a different seed gives a different S, and S A by
    the oracle's route equals the explicit product for dense and CSR A."""
    import scipy.sparse as sp
    s, m = 40, 20000
    S = rng.gaussian_sketch(5, s, m)
    N = S.size
    assert abs(S.mean()) < 6 * (1 / math.sqrt(s)) / math.sqrt(N)
    var = S.var() * s
    assert abs(var - 1.0) < 6 * math.sqrt(2.0 / N)
    col = (S ** 2).sum(axis=0)  # chi-square(s) / s per column: mean 1, variance 2/s
    assert abs(col.mean() - 1.0) < 6 * math.sqrt(2.0 / s / m)
    np.testing.assert_array_equal(rng.gaussian_sketch(5, s, 500), S[:, :500])
    assert np.mean(rng.gaussian_sketch(6, s, 500) != S[:, :500]) > 0.99
    r = np.random.default_rng(1)
    A = sp.random(300, 30, density=0.1, random_state=2, format="csr")
    Sg = rng.gaussian_sketch(9, 12, 300)
    np.testing.assert_allclose((A.T @ Sg.T).T, Sg @ A.toarray(), rtol=1e-13, atol=1e-13)
