"""Synthetic least-squares problems (inputs only; no method arithmetic).

Families follow the test sets of Sec. 6.3 of the paper and the five
benchmark workloads used by this project:

* ``haar``            -- Haar-distributed orthonormal columns (QR of a Gaussian
                         with the signs of diag(R) folded in; Mezzadri 2007).
* ``dense_svd``       -- A = U diag(sigma) V^T with Haar U, V (dense incoherent
                         family of Sec. 6.3.2).
* ``sparse_scaled``   -- CSR with a fixed number of distinct uniformly random
                         columns per row, N(0,1) values, column j scaled by
                         10^(-decades * j / (n - 1)).
* ``rbf_kernel``      -- Gaussian RBF kernel matrix exp(-||p_i - p_j||^2 / (2 h^2))
                         on points uniform in [0,1]^d.
* ``consistent_x``    -- b = A x* + e with e orthogonal to range(A) (Sec. 6.3.1).
* ``workload(c, ...)`` -- workload c in 1..5 at full or reduced size.

Seeds: numpy ``Generator(PCG64(1000 c + k))``, k = 0 for A, 1 for B,
2 for points / problem sizes.
"""
import math

import numpy as np
import scipy.sparse as sp

__all__ = ["rng_for", "haar", "dense_svd", "sparse_scaled", "rbf_kernel", "rbf_kernel_gpu", "consistent_x",
           "workload", "batch_shapes", "Workload", "dense_svd_gpu", "paper_sigma", "paper_dense_gpu",
           "paper_sparse"]


def rng_for(c, k):
    return np.random.Generator(np.random.PCG64(1000 * c + k))


def haar(rng, m, n):
    G = rng.standard_normal((m, n))
    Q, R = np.linalg.qr(G)
    return Q * np.where(np.diag(R) < 0, -1.0, 1.0)


def dense_svd(rng, m, n, sigma):
    U = haar(rng, m, n)
    V = haar(rng, n, n)
    return (U * sigma) @ V.T


def sparse_scaled(rng, m, n, per_row, decades):
    """CSR m x n, ``per_row`` distinct sorted uniform columns per row."""
    per_row = min(per_row, n)
    cols = np.empty((m, per_row), dtype=np.int64)
    pending = np.arange(m)
    while pending.size:
        draw = rng.integers(0, n, size=(pending.size, per_row))
        srt = np.sort(draw, axis=1)
        ok = np.all(srt[:, 1:] != srt[:, :-1], axis=1) if per_row > 1 else np.ones(pending.size, bool)
        cols[pending[ok]] = srt[ok]
        pending = pending[~ok]
    vals = rng.standard_normal((m, per_row))
    scale = 10.0 ** (-decades * np.arange(n) / max(n - 1, 1))
    vals = vals * scale[cols]
    indptr = np.arange(0, m * per_row + 1, per_row, dtype=np.int64)
    return sp.csr_matrix((vals.reshape(-1), cols.reshape(-1), indptr), shape=(m, n))


def rbf_kernel(rng, npts, dim=8, h=1.0, dtype=np.float32):
    P = rng.random((npts, dim))
    sq = np.sum(P * P, axis=1)
    D2 = np.maximum(sq[:, None] + sq[None, :] - 2.0 * (P @ P.T), 0.0)
    return np.exp(-D2 / (2.0 * h * h)).astype(dtype)


def consistent_x(rng, A, noise=0.0):
    """b = A x* + e, x* ~ N(0, I), e ~ noise * N(0, I) projected off range(A) twice."""
    Ad = A.toarray() if sp.issparse(A) else np.asarray(A, dtype=np.float64)
    m, n = Ad.shape
    xs = rng.standard_normal(n)
    b = Ad @ xs
    if noise > 0.0:
        Q, _ = np.linalg.qr(Ad)
        e = rng.standard_normal(m)
        for _ in range(2):
            e = e - Q @ (Q.T @ e)
        b = b + noise * e / np.linalg.norm(e)
    return xs, b


class Workload:
    def __init__(self, name, A, B, mu, block, tol, dtype):
        self.name, self.A, self.B, self.mu, self.block, self.tol, self.dtype = \
            name, A, B, mu, block, tol, dtype

    def __repr__(self):
        return f"Workload({self.name}, A{self.A.shape}, B{self.B.shape}, mu={self.mu}, b={self.block})"


def batch_shapes(count=64, seed_c=4, m_range=(5000, 100000), n_range=(500, 5000)):
    """Sizes of the batched workload: m ~ U{m_lo..m_hi}, then
    n ~ U{n_lo..min(n_hi, floor(m/4))}, decay k ~ U[2, 8]."""
    rng = rng_for(seed_c, 2)
    out = []
    for _ in range(count):
        m = int(rng.integers(m_range[0], m_range[1] + 1))
        n = int(rng.integers(n_range[0], min(n_range[1], m // 4) + 1))
        k = float(rng.uniform(2.0, 8.0))
        out.append((m, n, k))
    return out


def workload(c, scale=1.0):
    """Workload c (1..5).  ``scale`` < 1 shrinks m and n for tests.

    1: dense FP64 2000 x 200, sigma_i = 10^(-6 i / 200), consistent-x with
       1e-6 Gaussian noise, mu = 0, block 20, tol 1e-10.
    2: CSR 200000 x 20000, 10 non-zeros per row, column scaling logspace(0,-6),
       b ~ N(0,1), mu = 1e-4, block 100, tol 1e-8.
    3: RBF kernel (h = 1) on 40000 points in [0,1]^8, FP32, 16 RHS, mu = 1e-3,
       block 250, tol 1e-8.
    4: see ``batch_shapes`` (one problem per call is built by ``batch_problem``).
    5: dense FP32 100000 x 2000, sigma_i = 10^(-5 i / 2000), 32 RHS, mu = 1e-5,
       block 100, tol 1e-8.
    """
    ra, rb = rng_for(c, 0), rng_for(c, 1)
    if c == 1:
        m, n = max(8, int(2000 * scale)), max(4, int(200 * scale))
        sigma = 10.0 ** (-6.0 * np.arange(1, n + 1) / n)
        A = dense_svd(ra, m, n, sigma)
        xs = rb.standard_normal(n)
        b = A @ xs + 1e-6 * rb.standard_normal(m)
        return Workload("dense-svd-2000x200", A, b, 0.0, max(2, int(20 * scale)), 1e-10, "f64")
    if c == 2:
        m, n = max(16, int(200000 * scale)), max(8, int(20000 * scale))
        A = sparse_scaled(ra, m, n, 10, 6.0)
        b = rb.standard_normal(m)
        return Workload("csr-200000x20000-nnz10", A, b, 1e-4, max(2, int(100 * scale)), 1e-8, "f64")
    if c == 3:
        npts = max(16, int(40000 * scale))
        A = rbf_kernel(rng_for(c, 2), npts)
        B = rb.standard_normal((npts, 16)).astype(np.float32)
        return Workload("rbf-kernel-40000", A, B, 1e-3, max(2, int(250 * scale)), 1e-8, "f32")
    if c == 5:
        m, n = max(16, int(100000 * scale)), max(8, int(2000 * scale))
        sigma = 10.0 ** (-5.0 * np.arange(1, n + 1) / n)
        A = dense_svd(ra, m, n, sigma).astype(np.float32)
        B = rb.standard_normal((m, 32)).astype(np.float32)
        return Workload("dense-svd-100000x2000-adjoint", A, B, 1e-5, max(2, int(100 * scale)), 1e-8, "f32")
    raise ValueError(f"workload {c}: use batch_shapes/batch_problem for the batched workload")


def batch_problem(idx, m, n, k, nrhs=8, dtype=np.float32):
    """Problem ``idx`` of the batched workload (dense FP32, Haar factors)."""
    r = np.random.Generator(np.random.PCG64(4000 + 17 * idx + 3))
    sigma = 10.0 ** (-k * np.arange(1, n + 1) / n)
    A = dense_svd(r, m, n, sigma).astype(dtype)
    B = r.standard_normal((m, nrhs)).astype(dtype)
    return A, B


def dense_svd_gpu(seed, m, n, decades, nrhs, dtype="float32"):
    """Dense A = U diag(10^(-decades i / n)) V^T (Haar U, V from QR of
    Gaussians) and B (m x nrhs, N(0,1)) generated on the GPU with torch
    (seeded; for the large batched and adjoint workloads, where host QR is too
    slow).  Returns (A, B) as CUDA tensors, A in `dtype`, B in float64."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(int(seed))
    U, _ = torch.linalg.qr(torch.randn(m, n, device="cuda", dtype=torch.float64, generator=g))
    V, _ = torch.linalg.qr(torch.randn(n, n, device="cuda", dtype=torch.float64, generator=g))
    sig = 10.0 ** (-float(decades) * torch.arange(1, n + 1, device="cuda", dtype=torch.float64) / n)
    A = ((U * sig) @ V.T).to(getattr(torch, dtype)).contiguous()
    B = torch.randn(m, nrhs, device="cuda", dtype=torch.float64, generator=g)
    return A, B



def rbf_kernel_gpu(seed, npts, nrhs, dim=8, h=1.0):
    """Workload 3 generated on the GPU with torch (seeded): points uniform in
    [0,1]^dim, A_ij = exp(-||p_i - p_j||^2 / (2 h^2)) formed in FP64 and stored
    in FP32, B (npts x nrhs) N(0,1) in FP64.  Returns CUDA tensors (A, B)."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(int(seed))
    P = torch.rand(npts, dim, device="cuda", dtype=torch.float64, generator=g)
    sq = (P * P).sum(dim=1)
    A = torch.empty(npts, npts, device="cuda", dtype=torch.float32)
    step = 4096
    for i0 in range(0, npts, step):
        blk = P[i0:i0 + step]
        d2 = (sq[i0:i0 + step, None] + sq[None, :] - 2.0 * (blk @ P.T)).clamp_min_(0.0)
        A[i0:i0 + step] = torch.exp(-d2 / (2.0 * h * h)).to(torch.float32)
    B = torch.randn(npts, nrhs, device="cuda", dtype=torch.float64, generator=g)
    return A, B


# ---------------------------------------------------------------- the paper's test sets (Sec. 6.3)
def paper_sigma(n, decay):
    """Singular values of the paper's test matrices (largest first):
    'sharp7'  [logspace(2, -2, 0.2n), logspace(-4.8, -5, 0.8n)]  (kappa 1e7);
    'sharp15' [logspace(2, -2, 0.2n), logspace(-12, -13, 0.8n)]  (kappa 1e15);
    'smooth'  10^(2 - 15 sqrt((i - 1)/(n - 1))), i = 1..n: a root-exponential
              decay with kappa 1e15 (the text gives the type and kappa only;
              this law is a reading)."""
    if decay == "smooth":
        return 10.0 ** (2.0 - 15.0 * np.sqrt(np.arange(n) / max(n - 1, 1)))
    k = int(round(0.2 * n))
    lo = {"sharp7": (-4.8, -5.0), "sharp15": (-12.0, -13.0)}[decay]
    return np.concatenate([np.logspace(2, -2, k), np.logspace(lo[0], lo[1], n - k)])


def paper_dense_gpu(seed, m, n, decay, coherent=False, noise=0.0):
    """Dense test matrix A = U diag(sigma) V^T of Sec. 6.3.2 generated on the
    GPU (FP64, torch, seeded): incoherent U, V from QR of Gaussians (Haar), or
    coherent U = orth([I_n; 0] + 1e-8 J), V = orth(I_n + 1e-8 J) (J all ones);
    and a consistent-x right-hand side b = A x* + e, x* ~ N(0, I), e Gaussian
    projected off range(A) twice and scaled to noise ||A x*|| (the noise level
    is read as relative).  Returns CUDA tensors (A, b)."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(int(seed))
    dev, f64 = "cuda", torch.float64
    if coherent:
        U0 = torch.full((m, n), 1e-8, device=dev, dtype=f64)
        U0[:n, :n] += torch.eye(n, device=dev, dtype=f64)
        V0 = torch.full((n, n), 1e-8, device=dev, dtype=f64) + torch.eye(n, device=dev, dtype=f64)
    else:
        U0 = torch.randn(m, n, device=dev, dtype=f64, generator=g)
        V0 = torch.randn(n, n, device=dev, dtype=f64, generator=g)
    U, _ = torch.linalg.qr(U0)
    V, _ = torch.linalg.qr(V0)
    sig = torch.as_tensor(paper_sigma(n, decay), device=dev, dtype=f64)
    A = ((U * sig) @ V.T).contiguous()
    xs = torch.randn(n, device=dev, dtype=f64, generator=g)
    b = A @ xs
    if noise > 0.0:
        e = torch.randn(m, device=dev, dtype=f64, generator=g)
        for _ in range(2):
            e = e - U @ (U.T @ e)
        b = b + noise * float(b.norm()) * e / e.norm()
    return A, b


def paper_sparse(seed, m, n, decay, coherent=False, density=0.01):
    """Sparse test matrix of Sec. 6.3.2: B with ~density m n N(0,1) entries at
    uniform positions, C~ = D^f B with D = diag(N(0,1)) (f = 0 incoherent, 20
    coherent), columns of C~ normalised, A = C diag(sigma); b ~ N(0, I).
    Returns (scipy CSR A, b) on the host."""
    rng = np.random.Generator(np.random.PCG64(int(seed)))
    B = sp.random(m, n, density=density, format="csr", random_state=rng, data_rvs=rng.standard_normal)
    if coherent:
        d = rng.standard_normal(m) ** 20
        B = sp.diags(d) @ B
    norms = np.sqrt(np.asarray(B.multiply(B).sum(axis=0))).ravel()
    norms[norms == 0] = 1.0
    A = (B @ sp.diags(paper_sigma(n, decay) / norms)).tocsr()
    A.sort_indices()
    return A, rng.standard_normal(m)
