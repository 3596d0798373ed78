"""One LSQR phase on the augmented, right-preconditioned problem -- test infrastructure.

Follows Sec. 2.2 (LSQR = Golub-Kahan bidiagonalisation with a Givens QR of the
bidiagonal, Paige & Saunders 1982, Sec. 4 of that paper) applied to

    A~ = A_mu P^{-1},   A_mu = [A; delta I],   rhs r0 = b_aug - A_mu x

with the warm start of Sec. 3.2 (x <- x + P^{-1} y after the phase) and the
dynamic stopping rule of Sec. 5.3.2.  The left vector u is kept explicitly
augmented (m + n entries), because A_mu P^{-1} has no [A~; delta I] form.

Readings (where the text leaves a choice):
* delta = sqrt(mu): the objective weight mu of Sec. 1 enters A_mu as sqrt(mu).
* cvgrate_j = log(phibar_{j-1}/phibar_j), cvgdiff_j = phibar_{j-1} - phibar_j
  with phibar_0 = beta_1; the dynamic rule is tested from j = 2 on, a zero
  rate counts as an infinite ratio, and the rule is off in the final phase.
* "standard LSQR criteria" = Paige-Saunders test ||A~^T r|| <= eps ||A~||_F ||r||
  (running Frobenius estimate) or ||r|| <= eps ||b_aug||, plus the certified
  normal-equation bound  ||P|| ||A~^T r|| <= tol_ne ||A^T b||.
"""
import math

import numpy as np

STOP_NONE, STOP_METRIC, STOP_LSQR, STOP_DYNAMIC, STOP_BUDGET, STOP_EXACT = range(6)


def plsqr_phase(A, delta, b, x, pinv, *, nu=math.inf, sigma_l=0.0, eps_lsqr=1e-10,
                tol_ne=1e-8, atb_norm=1.0, pnorm=1.0, baug_norm=1.0, max_iter=10**9,
                history=None, pinv_t=None):
    """Run one warm-started PLSQR phase; returns (x_new, iterations, reason).

    ``pinv(z)`` applies P^{-1}; ``pinv_t(z)`` applies P^{-T} (None: P is
    symmetric and ``pinv`` serves for both); ``pinv=None`` means P = I
    (plain LSQR).
    """
    if pinv is None:
        pinv = lambda z: z  # noqa: E731
    if pinv_t is None:
        pinv_t = pinv
    m, n = A.shape
    aug = delta > 0.0
    u_t = b - A @ x
    u_b = -delta * x if aug else np.zeros(0)
    beta = math.sqrt(float(u_t @ u_t) + float(u_b @ u_b))
    if beta == 0.0:
        return x.copy(), 0, STOP_EXACT
    u_t = u_t / beta
    u_b = u_b / beta
    g = A.T @ u_t + (delta * u_b if aug else 0.0)
    v = pinv_t(g)
    alpha = math.sqrt(float(v @ v))
    if alpha == 0.0:
        return x.copy(), 0, STOP_EXACT
    v = v / alpha
    w = v.copy()
    y = np.zeros(n)
    phibar, rhobar = beta, alpha
    anorm2 = alpha * alpha
    phibar_prev = beta
    rate1 = None
    reason = STOP_BUDGET
    j = 0
    while j < max_iter:
        j += 1
        # bidiagonalisation: beta u = A~ v - alpha u ; alpha v = A~^T u - beta v
        t = pinv(v)
        u_t = A @ t - alpha * u_t
        u_b = (delta * t - alpha * u_b) if aug else u_b
        beta = math.sqrt(float(u_t @ u_t) + float(u_b @ u_b))
        if beta > 0.0:
            u_t = u_t / beta
            u_b = u_b / beta
            g = A.T @ u_t + (delta * u_b if aug else 0.0)
            v = pinv_t(g) - beta * v
            alpha = math.sqrt(float(v @ v))
            if alpha > 0.0:
                v = v / alpha
        else:
            alpha = 0.0
        anorm2 += alpha * alpha + beta * beta
        # Givens rotation eliminating beta from the lower bidiagonal
        rho = math.hypot(rhobar, beta)
        c, s = rhobar / rho, beta / rho
        theta = s * alpha
        rhobar = -c * alpha
        phi = c * phibar
        phibar = s * phibar
        y = y + (phi / rho) * w
        w = v - (theta / rho) * w
        if history is not None:
            history.append(phibar)
        # stopping tests
        arnorm = phibar * alpha * abs(c)  # ||A~^T r_j||
        if beta == 0.0 or alpha == 0.0:
            reason = STOP_EXACT
            break
        if pnorm * arnorm <= tol_ne * atb_norm:
            reason = STOP_METRIC
            break
        if arnorm <= eps_lsqr * math.sqrt(anorm2) * phibar or phibar <= eps_lsqr * baug_norm:
            reason = STOP_LSQR
            break
        rate = math.log(phibar_prev / phibar) if phibar > 0.0 else math.inf
        if rate1 is None:
            rate1 = rate
        elif math.isfinite(nu):
            ratio = math.inf if rate <= 0.0 else rate1 / rate
            if ratio > nu or (phibar_prev - phibar) < sigma_l:
                reason = STOP_DYNAMIC
                break
        phibar_prev = phibar
    return x + pinv(y), j, reason
