"""Closed-form references (oracle side) -- test infrastructure.

* ``solve_dense_qr``: x_mu = argmin ||A x - b||^2 + mu ||x||^2 from a
  Householder-QR least-squares solve of the augmented problem
  [A; sqrt(mu) I] x ~ [b; 0] (Sec. 2.1).  APLICUR and plain LSQR reach this
  same point; preconditioning changes the iterates, not the solution.
* ``solve_normal``: the same point from a Cholesky solve of (A^T A + mu I),
  used as an independent second route on well-conditioned inputs.
* ``adjoint``: gradients of a loss L(X) through X = x_mu(A, B):
      Z = (A^T A + mu I)^{-1} G,   dL/dB = A Z,   dL/dA = R Z^T - (A Z) X^T,
  R = B - A X.  (Not in the paper: a derivation by implicit differentiation
  of the normal equations A^T(B - A X) = mu X; pinned by finite differences.)
"""
import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def _dense(A):
    return A.toarray() if sp.issparse(A) else np.asarray(A, dtype=np.float64)


def solve_dense_qr(A, b, mu):
    A = _dense(A)
    m, n = A.shape
    if mu > 0.0:
        Aa = np.vstack([A, math.sqrt(mu) * np.eye(n)])
        ba = np.concatenate([b, np.zeros((n,) + b.shape[1:])])
    else:
        Aa, ba = A, b
    Q, R = np.linalg.qr(Aa)
    return sla.solve_triangular(R, Q.T @ ba)


def solve_normal(A, b, mu):
    A = _dense(A)
    H = A.T @ A + mu * np.eye(A.shape[1])
    return sla.cho_solve(sla.cho_factor(H), A.T @ b)


def gram_solve(A, G, mu):
    """(A^T A + mu I)^{-1} G by Cholesky: the normal-equations route."""
    A = _dense(A)
    H = A.T @ A + mu * np.eye(A.shape[1])
    return sla.cho_solve(sla.cho_factor(H), G)


def adjoint(A, X, B, G, mu):
    """Returns (Z, dB, dA) for the loss gradient G = dL/dX (dense A)."""
    A = _dense(A)
    Z = solve_dense_qr_rhs_bottom(A, G, mu)
    AZ = A @ Z
    R = B - A @ X
    dA = R @ Z.T - AZ @ X.T if X.ndim == 2 else np.outer(R, Z) - np.outer(AZ, X)
    return Z, AZ, dA


def solve_dense_qr_rhs_bottom(A, G, mu):
    """Z = argmin || [A; delta I] Z - [0; G/delta] || = (A^T A + mu I)^{-1} G."""
    A = _dense(A)
    m, n = A.shape
    delta = math.sqrt(mu)
    Aa = np.vstack([A, delta * np.eye(n)])
    rhs = np.concatenate([np.zeros((m,) + G.shape[1:]), G / delta])
    Q, R = np.linalg.qr(Aa)
    return sla.solve_triangular(R, Q.T @ rhs)
