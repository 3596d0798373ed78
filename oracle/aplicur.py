"""APLICUR (Alg. 3) and plain damped LSQR, FP64 on the CPU -- test infrastructure.

``aplicur`` takes the steps of Alg. 3 in the paper's order:

  Initialise  A_mu = [A; delta I], b_aug = [b; 0]; S = sparsesign(ceil(1.1 b), m, 8);
              E_row = Y = S A; I = J = {}; d_cur = inf; x = 0.
  repeat
    Part 1    [I, J] = augmentCUR(...) (Alg. 7); C, U = A(I,J)^dagger, R;
              E_row = Y - Y(:,J) U R; rho = randomized 2-norm bound (Sec. 5.3.1).
    Part 2    [Q_R, T_R] = augmentQR(Q_R, T_R, A(I+,:)^T) (Alg. 9).
    Part 3    if d_cur/(rho - eps_cur) >= nu_prec or rho <= eps_cur:
                 P = CURPreconditioner Part 2 (Alg. 2, or the SVD-free Alg. 8
                 when mu = 0 and precond = "svdfree"); nu = inf in the final phase;
                 x = lsqr(A_mu, b_aug, P, x, eps_lsqr, nu)  (warm start, Sec. 3.2);
                 d_cur = rho - eps_cur.
  until rho <= eps_cur.

Readings (where the text leaves a choice): delta = sqrt(mu); s = ceil(1.1 b) capped at
m; eps_cur defaults to 30 sqrt(mu) (3e-7 when mu = 0, Sec. 8.3); the step is
also final when the rank reaches min(n, max_rank) or the residual is exhausted;
the final phase stops on the certified normal-equation bound (the
Paige-Saunders eps_lsqr test, whose running Frobenius estimate of ||A~|| grows
with the iteration count, is used only in intermediate phases); the requested
accuracy eta <= tol_ne (eta = ||A^T(b - A x) - mu x|| / ||A^T b||,
from a fresh FP64 residual) ends the solve as soon as it holds after a phase,
and after the final phase further warm-started phases with the final P run
until it holds (the iterative-refinement view of Sec. 3.2).
Several right-hand sides share the sketch, the CUR sequence and every P (none
of them reads b); each column runs its own LSQR phases, so the multi-RHS result
is column-by-column the single-RHS one.
"""
import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from . import rng
from .cur import (Preconditioner, SvdFreePreconditioner, augment_cur, augment_qr, t_c_factor,
                  core_and_residual, rho_estimate)
from .lsqr import STOP_BUDGET, plsqr_phase


@dataclass
class Options:
    block: int = 20
    seed: int = 7
    eps_cur: float = -1.0      # <= 0: default reading
    nu_prec: float = 10.0
    nu_lsqr: float = 100.0
    eps_lsqr: float = 1e-10
    tol_ne: float = 1e-8
    max_iter: int = 100000
    max_rank: int = 0          # <= 0: min(m, n)
    r_probes: int = 10
    xi: int = 8                # non-zeros per column of the sparse sign sketch (1..8)
    sketch: str = "sparse"     # "sparse" (sparse sign, the default) or "gaussian"
    schedule: int = 0          # 0 fully adaptive; 1 rank-adaptive single shot; 2 fixed-rank single shot
    precond: str = "svd"       # "svd" (Alg. 2) or "svdfree" (Alg. 8, mu = 0 only)
    svdfree_floor: bool = True  # Alg. 8 target max(rho, eps_cur); False: rho as printed
    tc: str = "chol"            # T_C when chol(C^T C) breaks down: "chol" undo the step, "sketched" sketched CholQR


@dataclass
class Trace:
    ranks: list = field(default_factory=list)       # ell after each Part 1
    rhos: list = field(default_factory=list)
    rebuild: list = field(default_factory=list)     # whether Part 3 ran
    phase_iters: list = field(default_factory=list)
    phase_reason: list = field(default_factory=list)
    etas: list = field(default_factory=list)        # true eta after each phase
    I: list = field(default_factory=list)
    J: list = field(default_factory=list)
    sigma_hat: list = field(default_factory=list)
    iters: int = 0


class RebuildRule:
    """The re-preconditioning test of Alg. 3, Part 3 (Sec. 5.3.2).

    A new preconditioner is built when the step is final (rho <= eps_cur, or
    the rank can grow no further), or when the CUR error has dropped enough
    since the last build: d_cur / (rho - eps_cur) >= nu_prec, where d_cur is
    rho - eps_cur at the last build (+inf before the first, so the first
    step always builds).  ``adaptive=False`` (the single-shot schedules of
    Sec. 7.1) builds at the final step only.
    """

    def __init__(self, eps_cur, nu_prec, adaptive=True):
        self.eps_cur = eps_cur
        self.nu_prec = nu_prec
        self.adaptive = adaptive
        self.d_cur = math.inf

    def __call__(self, rho, final):
        gap = rho - self.eps_cur
        rebuild = final or (self.adaptive and self.d_cur / gap >= self.nu_prec)
        if rebuild:
            self.d_cur = gap
        return rebuild


def default_eps_cur(mu):
    return 30.0 * math.sqrt(mu) if mu > 0.0 else 3e-7


def sketch_rows(block, m):
    return max(1, min(m, int(math.ceil(1.1 * block - 1e-12))))


def ne_residual(A, b, x, mu):
    """eta(x) = ||A^T(b - A x) - mu x|| / ||A^T b|| (0 when A^T b = 0)."""
    atb = float(np.linalg.norm(A.T @ b))
    if atb == 0.0:
        return 0.0
    return float(np.linalg.norm(A.T @ (b - A @ x) - mu * x)) / atb


def lsqr_plain(A, b, mu, tol_ne=1e-8, eps_lsqr=0.0, max_iter=100000, x0=None):
    """Plain damped LSQR on [A; sqrt(mu) I] (P = I), restarted from a fresh
    residual until eta <= tol_ne; returns (x, iterations)."""
    n = A.shape[1]
    delta = math.sqrt(mu)
    x = np.zeros(n) if x0 is None else x0.copy()
    atb = float(np.linalg.norm(A.T @ b))
    if atb == 0.0:
        return x, 0
    total = 0
    while total < max_iter:
        x, it, _ = plsqr_phase(A, delta, b, x, None, eps_lsqr=eps_lsqr, tol_ne=tol_ne,
                               atb_norm=atb, baug_norm=float(np.linalg.norm(b)),
                               max_iter=max_iter - total)
        total += it
        if ne_residual(A, b, x, mu) <= tol_ne or it == 0:
            break
    return x, total


def aplicur(A, b, mu, opts=None, trace=None):
    """Alg. 3 for one right-hand side; returns x (and fills ``trace``)."""
    opts = opts or Options()
    if b.ndim == 2:
        return np.column_stack([aplicur(A, b[:, k], mu, opts, trace if k == 0 else None)
                                for k in range(b.shape[1])])
    A = A.tocsr() if sp.issparse(A) else np.asarray(A, dtype=np.float64)
    m, n = A.shape
    delta = math.sqrt(mu)
    svdfree = opts.precond == "svdfree"
    if svdfree and mu != 0.0:
        # Sec. 3.1 defines the SVD-free variant for the unregularised problem;
        # its regularised form (a CUR of A_mu) is not built.
        raise ValueError("the SVD-free preconditioner needs mu = 0")
    eps_cur = opts.eps_cur if opts.eps_cur > 0 else default_eps_cur(mu)
    max_rank = min(m, n) if opts.max_rank <= 0 else min(opts.max_rank, m, n)
    # initialisation
    s = sketch_rows(opts.block, m)
    if opts.sketch == "gaussian":
        S = rng.gaussian_sketch(opts.seed, s, m)  # dense s x m
        Y = np.asarray((A.T @ S.T).T if sp.issparse(A) else S @ A, dtype=np.float64)
    else:
        S = rng.sparse_sign_matrix(opts.seed, s, m, opts.xi)
        Y = np.asarray((S @ A).toarray() if sp.issparse(A) else S @ A, dtype=np.float64)
    probes = rng.gaussian_probes(opts.seed, n, opts.r_probes)
    E_row = Y.copy()
    I = np.zeros(0, np.int64)
    J = np.zeros(0, np.int64)
    C = W = R = None
    Q_R = T_R = None
    rule = RebuildRule(eps_cur, opts.nu_prec, adaptive=opts.schedule == 0)
    x = np.zeros(n)
    atb = float(np.linalg.norm(A.T @ b))
    bnorm = float(np.linalg.norm(b))
    if atb == 0.0:
        return x
    total = 0
    eta = math.inf
    while True:
        # Part 1: update CUR
        # the rank cap also limits the last increment (reading: l never exceeds max_rank)
        I_plus, J_plus, exhausted = augment_cur(A, E_row, I, J, C, W, R, min(opts.block, max_rank - len(J)))
        if len(J_plus) == 0 and len(J) == 0:
            break
        prev = (I, J, C, W, R, E_row, Q_R, T_R, rho if len(J) else None)
        I = np.concatenate([I, I_plus])
        J = np.concatenate([J, J_plus])
        C, W, R, E_row = core_and_residual(A, Y, I, J)
        rho = rho_estimate(E_row, probes)
        # Part 2: update the QR factorisation of R^T
        if len(I_plus):
            Q_R, T_R = augment_qr(Q_R, T_R, A[I_plus, :].T)
        # T_C of Alg. 2: chol(C^T C); when C^T C is no longer positive
        # definite in floating point (new columns nearly dependent on C),
        # with tc = "sketched" the sketched Cholesky QR that Alg. 2 and Alg. 3
        # Part 3 name for stability.  Reading: when no T_C results, the step is
        # undone and treated as exhaustion.
        sk = opts.tc == "sketched"
        T_C = t_c_factor(C, opts.seed, sketched=sk)
        if T_C is None and len(prev[1]):
            I, J, C, W, R, E_row, Q_R, T_R, rho = prev
            T_C = t_c_factor(C, opts.seed, sketched=sk)
            exhausted = True
        # Sec. 7.1 variants: single shot builds P once, at the final rank
        # (schedule 2: the rank cap, whatever rho)
        grown = exhausted or len(J) >= max_rank
        final = grown or (opts.schedule != 2 and rho <= eps_cur)
        if trace is not None:
            trace.ranks.append(len(J))
            trace.rhos.append(rho)
            trace.I, trace.J = I.copy(), J.copy()
        # Part 3: re-precondition and run LSQR
        rebuild = rule(rho, final)
        if trace is not None:
            trace.rebuild.append(rebuild)
        if rebuild:
            if svdfree:
                P = SvdFreePreconditioner(C, W, Q_R, T_R, rho, eps_cur, floor=opts.svdfree_floor, T_C=T_C)
                pinv_t = P.inv_t
            else:
                P = Preconditioner(C, W, Q_R, T_R, delta, T_C=T_C)
                pinv_t = None
            nu = math.inf if final else opts.nu_lsqr
            x, it, why = plsqr_phase(A, delta, b, x, P.inv, pinv_t=pinv_t, nu=nu, sigma_l=P.sigma_l,
                                     eps_lsqr=0.0 if final else opts.eps_lsqr,
                                     tol_ne=opts.tol_ne,
                                     atb_norm=atb, pnorm=P.pnorm, baug_norm=bnorm,
                                     max_iter=opts.max_iter - total)
            total += it
            eta = ne_residual(A, b, x, mu)
            if trace is not None:
                trace.phase_iters.append(it)
                trace.phase_reason.append(why)
                trace.etas.append(eta)
                trace.sigma_hat.append(P.target)
            if eta <= opts.tol_ne or total >= opts.max_iter:
                break
            if final:
                # refinement phases with the final P until the accuracy holds
                stalls = 0
                while eta > opts.tol_ne and total < opts.max_iter and stalls < 3:
                    eta_prev = eta
                    x, it, why = plsqr_phase(A, delta, b, x, P.inv, pinv_t=pinv_t, sigma_l=P.sigma_l,
                                             eps_lsqr=0.0, tol_ne=opts.tol_ne,
                                             atb_norm=atb, pnorm=P.pnorm, baug_norm=bnorm,
                                             max_iter=opts.max_iter - total)
                    total += it
                    eta = ne_residual(A, b, x, mu)
                    if trace is not None:
                        trace.phase_iters.append(it)
                        trace.phase_reason.append(why)
                        trace.etas.append(eta)
                    if it == 0 or why == STOP_BUDGET:
                        break
                    stalls = stalls + 1 if eta > 0.5 * eta_prev else 0
        if final:
            break
    if trace is not None:
        trace.iters = total
    return x
