"""Error bounds of the parity tests, derived from the arithmetic.

A computed x whose normal-equation residual is eta = ||A^T (b - A x) - mu x||
/ ||A^T b|| differs from the minimiser x* = (A^T A + mu I)^{-1} A^T b by

    x - x* = -(A^T A + mu I)^{-1} (A^T (b - A x) - mu x),
    ||x - x*|| <= eta ||A^T b|| / sigma_min(A_mu)^2,

with sigma_min(A_mu)^2 = sigma_min(A)^2 + mu.  A reference x* computed by a
backward-stable dense least-squares solver carries its own perturbation
floor, 10 (kappa u + kappa^2 u ||r|| / (||A_mu|| ||x||)) with kappa =
kappa(A_mu), u = 2^-53 and r the least-squares residual (Golub & Van Loan,
Thm. 5.3.1, with a factor 10 of slack for the solver's constants).  The
tests compare solutions against the sum of both terms; every check prints
the measured error beside its bound.
"""
import numpy as np
import scipy.sparse as sp

U64 = 2.0 ** -53


def _dense(A):
    return A.toarray() if sp.issparse(A) else np.asarray(A, dtype=np.float64)


def eta_of(A, b, x, mu):
    r = b - A @ x
    g = A.T @ r - mu * x
    atb = np.linalg.norm(A.T @ b)
    return float(np.linalg.norm(g) / atb) if atb > 0 else 0.0


def conditioning(A, mu):
    """(sigma_min, sigma_max) of A_mu = [A; sqrt(mu) I]."""
    s = np.linalg.svd(_dense(A), compute_uv=False)
    smin = float(np.sqrt(s[-1] ** 2 + mu)) if A.shape[0] >= A.shape[1] else float(np.sqrt(mu))
    return smin, float(np.sqrt(s[0] ** 2 + mu))


def solution_bound(A, b, mu, xref, etas):
    """Bound on ||x - xref|| / ||xref|| for solutions whose eta values are
    `etas` (one for each side that is not the dense reference)."""
    smin, smax = conditioning(A, mu)
    kappa = smax / smin
    xn = np.linalg.norm(xref)
    r = np.linalg.norm(np.concatenate([b - A @ xref, -np.sqrt(mu) * xref]))
    floor = 10.0 * (kappa * U64 + kappa ** 2 * U64 * r / (smax * xn))
    atb = np.linalg.norm(A.T @ b)
    return sum(etas) * atb / (smin ** 2 * xn) + floor


def check_solution(x, xref, A, b, mu, label="", other_etas=()):
    """Assert ||x - xref|| <= bound * ||xref||; returns (error, bound)."""
    x = np.asarray(x, dtype=np.float64)
    eta = eta_of(A, b, x, mu)
    bound = solution_bound(A, b, mu, xref, [eta, *other_etas])
    err = float(np.linalg.norm(x - xref) / np.linalg.norm(xref))
    print(f"[parity] {label}: ||x - x_ref||/||x_ref|| = {err:.3e} (bound {bound:.3e}, eta {eta:.2e})")
    assert err <= bound, f"{label}: error {err:.3e} above the bound {bound:.3e}"
    return err, bound
