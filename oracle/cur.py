"""CUR building blocks of APLICUR (oracle side) -- test infrastructure.

* ``lupp_pivots``     -- first k row pivots of LU with partial pivoting, the
                        selection rule of Alg. 7 (``lu(X,'vector')``).  Written
                        as the textbook right-looking elimination; pinned in the
                        tests against LAPACK getrf (scipy.linalg.lu_factor).
* ``augment_cur``     -- Alg. 7 (augmentCUR).
* ``core_and_residual`` -- C, U = A(I,J)^dagger, R and the sketched residual
                        E_row = Y - Y(:,J) U R of Alg. 3, Part 1.
* ``rho_estimate``    -- the randomized 2-norm bound of Sec. 5.3.1 with r probes.
* ``augment_qr``      -- Alg. 9 (block classical Gram-Schmidt with one
                        re-orthogonalisation, then QR of the remainder).
* ``Preconditioner``  -- Alg. 2, Part 2 (SVD-based CUR preconditioner, eq. of
                        Sec. 3.1 with target level sqrt(sigma_l^2 + delta^2)).
* ``sketched_cholqr``  -- T_C by sketched Cholesky QR (the stable choice Alg. 2
                        and Alg. 3 Part 3 name): the R factor of a Gaussian
                        sketch Theta C (two shifted and two plain Cholesky QR
                        passes), then one Cholesky QR of C R^{-1}.
* ``SvdFreePreconditioner`` -- Alg. 8 (SVD-free variant of Sec. 3.1 for mu = 0):
                        M^{-1} = T_R^{-T} A(I,J) T_C^{-1} by two triangular
                        solves, P~^{-1} = s Q_R M^{-1} Q_R^T + (I - Q_R Q_R^T)
                        with target level s = max(rho, eps_cur); not symmetric, so its
                        transpose is applied separately.

Readings: ties in the pivot search go to the first maximal entry in the
current row order (LAPACK idamax); a zero pivot column means the residual is
exhausted and selection stops there; E_col uses the factors from before the
augmentation (Alg. 7 forms it before the index sets are used to rebuild C, U, R).
"""
import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

RHO_CONST = 10.0 * math.sqrt(2.0 / math.pi)


def _dense(X):
    return X.toarray() if sp.issparse(X) else np.asarray(X, dtype=np.float64)


def lupp_pivots(X, k):
    """First ``k`` pivot rows of partial-pivoting LU of the r x c matrix X.

    Returns (pivots, k_eff): ``pivots`` are original row indices in pivot
    order; ``k_eff < k`` when a pivot column is identically zero.
    """
    X = np.array(_dense(X), dtype=np.float64, copy=True)
    r, c = X.shape
    k = min(k, r, c)
    order = np.arange(r)  # order[p] = original row now at position p
    for q in range(k):
        col = np.abs(X[q:, q])
        p = q + int(np.argmax(col))  # argmax returns the first maximum
        if col[p - q] == 0.0:
            return order[:q].copy(), q
        if p != q:
            X[[q, p], :] = X[[p, q], :]
            order[[q, p]] = order[[p, q]]
        l = X[q + 1:, q] / X[q, q]
        X[q + 1:, q] = l
        X[q + 1:, q + 1:] -= np.outer(l, X[q, q + 1:])
    return order[:k].copy(), k


def augment_cur(A, Y_res, I, J, C, W, R, block):
    """Alg. 7 (augmentCUR): choose up to ``block`` new column and row indices.

    ``Y_res`` is the current sketched residual E_row (s x n); ``C, W, R`` are
    A(:,J), A(I,J), A(I,:) of the current approximation (None when empty).
    Returns (I_plus, J_plus, exhausted).
    """
    m, n = A.shape
    s = Y_res.shape[0]
    ell = len(J)
    beff = min(block, n - ell, m - ell, s)
    if beff <= 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64), True
    E = np.array(Y_res, copy=True)
    if ell:
        E[:, J] = 0.0
    J_plus, k1 = lupp_pivots(E.T, beff)
    Acols = _dense(A[:, J_plus])
    if ell:
        # E_col = A(:,J+) - C U R(:,J+) with U = W^{-1} (pre-augmentation factors)
        UR = sla.lu_solve(sla.lu_factor(W), _dense(R[:, J_plus]))
        E_col = Acols - _dense(C @ UR)
        E_col[I, :] = 0.0
    else:
        E_col = Acols
    I_plus, k2 = lupp_pivots(E_col, k1)
    J_plus = J_plus[:k2]
    return I_plus, J_plus, (k2 < beff)


def core_and_residual(A, Y, I, J):
    """C, W = A(I,J), R and E_row = Y - Y(:,J) W^{-1} R (Alg. 3, Part 1)."""
    C = A[:, J]
    R = A[I, :]
    W = _dense(A[I, :][:, J])
    lu = sla.lu_factor(W)
    YJU = sla.lu_solve(lu, Y[:, J].T, trans=1).T  # Y(:,J) W^{-1}
    E_row = Y - _dense((sp.csr_matrix(YJU) @ R) if sp.issparse(R) else YJU @ R)
    return C, W, R, E_row


def rho_estimate(E_row, probes):
    """rho = 10 sqrt(2/pi) max_i ||E_row w_i|| (Sec. 5.3.1)."""
    return RHO_CONST * float(np.max(np.linalg.norm(E_row @ probes, axis=0)))


def augment_qr(Q, T, Cnew):
    """Alg. 9: QR of [Q T, Cnew] from the QR Q T of the old block."""
    Cnew = _dense(Cnew)
    if Q is None or Q.shape[1] == 0:
        Qe, Re = np.linalg.qr(Cnew)
        sg = np.where(np.diag(Re) < 0, -1.0, 1.0)
        return Qe * sg, Re * sg[:, None]
    P1 = Q.T @ Cnew
    E = Cnew - Q @ P1
    P2 = Q.T @ E
    E = E - Q @ P2
    Qe, Re = np.linalg.qr(E)
    sg = np.where(np.diag(Re) < 0, -1.0, 1.0)
    Qe, Re = Qe * sg, Re * sg[:, None]
    l, p = T.shape[0], Cnew.shape[1]
    Tn = np.zeros((l + p, l + p))
    Tn[:l, :l] = T
    Tn[:l, l:] = P1 + P2
    Tn[l:, l:] = Re
    return np.hstack([Q, Qe]), Tn


# Stream offset of the embedding Theta of sketched Cholesky QR: Theta is the
# Gaussian embedding of seed + TC_SEED_OFFSET (stream 3), so it never
# coincides with the Gaussian sketch of A.
TC_SEED_OFFSET = 7919
U64 = 2.0 ** -53


def _chol_upper(G):
    """Upper U with U^T U = G, or None when the Cholesky breaks down."""
    try:
        return np.linalg.cholesky(G).T
    except np.linalg.LinAlgError:
        return None


def sketched_cholqr(C, seed):
    """T_C (upper, positive diagonal, T_C^T T_C = C^T C to rounding) for a
    C (m x l) too ill-conditioned for chol(C^T C), or None when even this
    breaks down (the columns are dependent to working precision).

    Steps (sketched Cholesky QR, Balabanov 2022, with the sketch's own R
    factor by shifted Cholesky QR, Fukaya et al. 2020):
      Theta: k x m Gaussian embedding, k = min(m, 2 l);  X_0 = Theta C;
      two shifted passes  R_i = chol(X^T X + s I),  s = 11 (k l + l (l + 1)) u ||X||_F^2,
      then two plain passes  R_i = chol(X^T X);  each pass X <- X R_i^{-1};
      R = R_4 R_3 R_2 R_1 (the R factor of Theta C);
      Q = C R^{-1};  R' = chol(Q^T Q);  T_C = R' R.
    One shifted pass brings cond(X) to about sqrt(cond(X_0) / sqrt(u)); the
    second makes the plain passes safe up to cond(C) near 1/u.
    """
    from oracle import rng
    C = _dense(C)
    m, l = C.shape
    k = min(m, 2 * l)
    X = rng.gaussian_sketch(seed + TC_SEED_OFFSET, k, m) @ C
    R = np.eye(l)
    for shifted in (True, True, False, False):
        shift = 11.0 * (k * l + l * (l + 1)) * U64 * float(np.sum(X * X)) if shifted else 0.0
        Ri = _chol_upper(X.T @ X + shift * np.eye(l))
        if Ri is None:
            return None
        X = sla.solve_triangular(Ri, X.T, trans=1, lower=False).T
        R = Ri @ R
    Q = sla.solve_triangular(R, C.T, trans=1, lower=False).T
    Rp = _chol_upper(Q.T @ Q)
    if Rp is None:
        return None
    return np.triu(Rp @ R)


def t_c_factor(C, seed, sketched=True):
    """T_C of Alg. 2: chol(C^T C) when it exists, else (sketched) sketched
    Cholesky QR; None when what was tried breaks down."""
    CtC = C.T @ C
    T = _chol_upper(CtC.toarray() if sp.issparse(CtC) else np.asarray(CtC))
    if T is None and sketched:
        T = sketched_cholqr(C, seed)
    return T


class Preconditioner:
    """SVD-based CUR preconditioner (Alg. 2, Part 2; Sec. 3.1).

    P = sigma^{-1} V Lam V^T + (I - V V^T),  Lam = sqrt(Sigma^2 + delta^2),
    sigma = sqrt(sigma_l^2 + delta^2), built from T_C = chol(C^T C),
    M = T_C U T_R^T = U_M Sigma V_M^T and V = Q_R V_M.
    """

    def __init__(self, C, W, Q_R, T_R, delta, T_C=None):
        if T_C is None:
            T_C = np.linalg.cholesky(_dense(C.T @ C)).T  # upper, T_C^T T_C = C^T C
        M = T_C @ sla.lu_solve(sla.lu_factor(W), T_R.T)
        _, sig, VmT = np.linalg.svd(M)
        self.sigma = sig
        self.V = Q_R @ VmT.T
        self.Lam = np.sqrt(sig ** 2 + delta ** 2)
        self.target = math.sqrt(sig[-1] ** 2 + delta ** 2)
        self.d = self.target / self.Lam - 1.0
        self.sigma_l = float(sig[-1])  # unregularised smallest singular value
        self.pnorm = max(1.0, float(self.Lam[0]) / self.target)

    def inv(self, z):
        """P^{-1} z = z + V ((sigma/Lam - 1) * (V^T z)); P is symmetric."""
        return z + self.V @ (self.d * (self.V.T @ z))

    def dense_inverse(self):
        n = self.V.shape[0]
        return np.eye(n) + (self.V * self.d) @ self.V.T


class SvdFreePreconditioner:
    """SVD-free CUR preconditioner (Alg. 8; the SVD-free variant of Sec. 3.1),
    defined for mu = 0.

    T_C = chol(C^T C) (upper), [Q_R, T_R] the QR of R^T with a positive
    diagonal of T_R (the factorisation is then unique; P~ depends on the sign
    convention, its singular values do not), M^{-1} = T_R^{-T} W T_C^{-1} with
    W = A(I,J), and

        P~^{-1}   = target Q_R M^{-1}   Q_R^T + (I - Q_R Q_R^T),
        P~^{-T}   = target Q_R M^{-T}   Q_R^T + (I - Q_R Q_R^T),

    with target = max(rho, eps_cur): rho is the CUR error estimate (Alg. 8
    takes the estimate of Sec. 5.3.1 as the target level).  Readings: the
    target is not taken below the requested CUR accuracy eps_cur, so the
    final build (reached when rho <= eps_cur) uses eps_cur.  The literal
    level flattens the captured spectrum to a rho far below the requested
    accuracy, and ||P~|| = ||M|| / rho then makes the certified stop much
    stricter than the normal-equation residual needs (more than three times
    the iterations on the sparse sharp kappa = 1e15 set; ``floor=False``
    keeps it for that comparison); rho = 0, an exact CUR, would make
    P~^{-1} singular.  The dynamic rule's smallest resolved singular value
    is taken as the target; ||P~|| = max(1, ||M|| / target) is bounded
    above by the Frobenius norm of M = T_C W^{-1} T_R^T.
    """

    def __init__(self, C, W, Q_R, T_R, rho, eps_cur, floor=True, T_C=None):
        if T_C is None:
            T_C = np.linalg.cholesky(_dense(C.T @ C)).T
        sg = np.where(np.diag(T_R) < 0, -1.0, 1.0)
        self.Q = Q_R * sg
        T_R = T_R * sg[:, None]
        W = _dense(W)
        # M^{-1} = T_R^{-T} (W T_C^{-1})
        WTi = sla.solve_triangular(T_C, W.T, trans=1, lower=False).T  # W T_C^{-1}
        self.Minv = sla.solve_triangular(T_R, WTi, trans=1, lower=False)
        M = T_C @ np.linalg.solve(W, T_R.T)
        # floor=False: the literal Alg. 8 level (rho itself), kept for the
        # test that compares the two readings
        self.target = max(float(rho), float(eps_cur)) if floor else float(rho)
        self.sigma_l = self.target
        self.pnorm = max(1.0, float(np.linalg.norm(M, "fro")) / self.target)
        self.T_R = T_R

    def inv(self, z):
        """P~^{-1} z = z + Q_R (target M^{-1} - I) Q_R^T z."""
        c = self.Q.T @ z
        return z + self.Q @ (self.target * (self.Minv @ c) - c)

    def inv_t(self, z):
        """P~^{-T} z = z + Q_R (target M^{-T} - I) Q_R^T z."""
        c = self.Q.T @ z
        return z + self.Q @ (self.target * (self.Minv.T @ c) - c)

    def dense_inverse(self):
        n = self.Q.shape[0]
        H = self.target * self.Minv - np.eye(self.Minv.shape[0])
        return np.eye(n) + self.Q @ H @ self.Q.T
