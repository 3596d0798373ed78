"""Counter-based random stream of the method (oracle side) -- test infrastructure.

The method draws two kinds of random numbers:

* the sparse sign embedding S (Definition 5.1, used once in Alg. 3 to form
  Y = S A): every column of S has xi' = min(8, s) non-zeros at distinct
  uniformly random rows, each an independent Rademacher sign, scaled by
  1/sqrt(xi');
* r = 10 standard Gaussian probe vectors w_i of the randomized 2-norm bound
  that defines rho (Sec. 5.3.1).

Both sides (this oracle and the HIP library) implement the same generator
from its published definition, so that S is bit-identical:

  SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
  generators", OOPSLA 2014): state += 0x9E3779B97F4A7C15, output
  mix64(state), with mix64 the variant-13 finalizer
      z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
      z = (z ^ (z >> 27)) * 0x94D049BB133111EB
      z =  z ^ (z >> 31)            (all arithmetic mod 2^64).

Stream layout (all counters 0-based):
  key(seed, stream)      = mix64(seed + G * (stream + 1))
  draw(seed, stream, c)  = mix64(key(seed, stream) + G * (c + 1)),  G = 0x9E37...
  stream 0: row of non-zero t of column i, attempt a: c = (8 i + t) * 64 + a,
            row = draw mod s, redrawn (a += 1) while it repeats an earlier row
            of the same column; after 64 attempts the smallest unused row.
  stream 1: sign of non-zero t of column i: c = 8 i + t, negative iff the top
            bit of the draw is set.
  stream 2: probe entry (j, i) (component j of vector i): c = i n + j,
            Box-Muller with u1 = ((d0 >> 11) + 1) 2^-53, u2 = (d1 >> 11) 2^-53
            where d0 = draw(2c), d1 = draw(2c + 1):
            z = sqrt(-2 ln u1) cos(2 pi u2).
  stream 3: Gaussian sketch entry (h, i): c = i s + h, the same Box-Muller,
            divided by sqrt(s).
"""
import math

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
MAX_ATTEMPTS = 64


def mix64(z):
    """SplitMix64 output finalizer on uint64 arrays (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def key(seed, stream):
    with np.errstate(over="ignore"):
        return mix64(np.uint64(seed) + GOLDEN * np.uint64(stream + 1))


def draw(seed, stream, ctr):
    """Output number ``ctr`` of the SplitMix64 sequence keyed by (seed, stream)."""
    k = key(seed, stream)
    ctr = np.asarray(ctr, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(k + GOLDEN * (ctr + np.uint64(1)))


def sketch_nnz(s, xi=8):
    """xi' = min(xi, s): non-zeros per column of S (Alg. 3 initialisation,
    App. B.3; the paper's default xi = 8).  The counters below give each
    column 8 slots, so 1 <= xi <= 8."""
    if not 1 <= xi <= 8:
        raise ValueError("xi must be in [1, 8]")
    return min(xi, s)


def sparse_sign(seed, s, m, xi=8):
    """Sparse sign embedding S in R^{s x m} (Definition 5.1) with min(xi, s)
    non-zeros per column.

    Returns (rows, signs, xi'): ``rows[i, t]`` is the row of non-zero t of
    column i (distinct within a column), ``signs[i, t]`` is +-1, and each
    non-zero equals signs / sqrt(xi').
    """
    xi = sketch_nnz(s, xi)
    rows = np.full((m, xi), -1, dtype=np.int64)
    cols = np.arange(m, dtype=np.uint64)
    for t in range(xi):
        pending = np.ones(m, dtype=bool)
        for a in range(MAX_ATTEMPTS):
            idx = np.nonzero(pending)[0]
            if idx.size == 0:
                break
            c = (np.uint64(8) * cols[idx] + np.uint64(t)) * np.uint64(64) + np.uint64(a)
            h = (draw(seed, 0, c) % np.uint64(s)).astype(np.int64)
            clash = np.zeros(idx.size, dtype=bool)
            for tp in range(t):
                clash |= rows[idx, tp] == h
            ok = ~clash
            rows[idx[ok], t] = h[ok]
            pending[idx[ok]] = False
        # fall-back: smallest unused row (reached with probability < 1e-15)
        for i in np.nonzero(pending)[0]:
            used = set(rows[i, :t].tolist())
            rows[i, t] = next(r for r in range(s) if r not in used)
    c = np.uint64(8) * cols[:, None] + np.arange(xi, dtype=np.uint64)[None, :]
    top = draw(seed, 1, c) >> np.uint64(63)
    signs = np.where(top == 0, 1.0, -1.0)
    return rows, signs, xi


def sparse_sign_matrix(seed, s, m, xi=8):
    """S as a scipy CSR matrix (s x m)."""
    import scipy.sparse as sp
    rows, signs, xi = sparse_sign(seed, s, m, xi)
    cols = np.repeat(np.arange(m), xi)
    vals = signs.reshape(-1) / np.sqrt(xi)
    return sp.csr_matrix((vals, (rows.reshape(-1), cols)), shape=(s, m))


def gaussian_sketch(seed, s, m):
    """Gaussian embedding S in R^{s x m} with i.i.d. N(0, 1/s) entries (the
    Gaussian sketch of Sec. 5.1 / App. B.3): entry (h, i) is a Box-Muller
    normal of the stream-3 draws 2c and 2c + 1, c = i s + h (column-major
    order, so the first m columns do not depend on m), divided by sqrt(s)."""
    h = np.arange(s, dtype=np.uint64)[:, None]
    i = np.arange(m, dtype=np.uint64)[None, :]
    c = i * np.uint64(s) + h
    d0 = draw(seed, 3, np.uint64(2) * c)
    d1 = draw(seed, 3, np.uint64(2) * c + np.uint64(1))
    u1 = ((d0 >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = (d1 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2) / math.sqrt(s)


def gaussian_probes(seed, n, r):
    """r standard Gaussian probe vectors as the columns of an n x r array (Sec. 5.3.1)."""
    i = np.arange(r, dtype=np.uint64)[None, :]
    j = np.arange(n, dtype=np.uint64)[:, None]
    c = i * np.uint64(n) + j
    d0 = draw(seed, 2, np.uint64(2) * c)
    d1 = draw(seed, 2, np.uint64(2) * c + np.uint64(1))
    u1 = ((d0 >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = (d1 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
