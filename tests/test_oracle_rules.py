"""Hand-worked pins of the oracle's decision rules (Sec. 5.3.2, Alg. 3 Part 3,
Alg. 8's target level).

The dynamic stopping rule and the re-preconditioning test change iteration
counts and rebuild points but not the solution, so solution tests cannot catch
a mistake in them (a swapped ratio, phibar_0 off by one, a sign slip in the
CUR gap).  These cases fix them from values worked out by hand.

Dynamic rule, worked case.  A = diag(1, 2, 3), b = (1, 1, 1), x0 = 0, mu = 0,
no preconditioner.  After j LSQR steps the residual is the part of b
orthogonal to A K_j(A^T A, A^T b) = span{lam^k * b : k = 1..j} with
lam = (1, 4, 9) (elementwise powers), so
  phibar_0 = ||b|| = sqrt(3),
  phibar_1^2 = 3 - (sum lam)^2 / sum lam^2 = 3 - 14^2/98 = 1,
  phibar_2 = |b . n| / ||n|| with n = (1,4,9) x (1,16,81) / 12 = (15, -6, 1):
             10 / sqrt(262) = sqrt(50/131) = 0.61780206...,
  phibar_3 = 0 (three distinct singular values).
Rates: cvgrate_1 = log(phibar_0/phibar_1) = log sqrt(3) = 0.549306...,
       cvgrate_2 = log(phibar_1/phibar_2) = 0.481576...,
so cvgrate_1/cvgrate_2 = 1.140616... and cvgdiff_2 = phibar_1 - phibar_2 =
0.382198....  The rule is first tested at j = 2.  With nu = 1.1 it fires at
j = 2; with nu = 1.2 it does not.  The swapped ratio (0.877) and a rate_1
taken from phibar_1/phibar_2 (ratio 1) would not fire at nu = 1.1.  With
sigma_l = 0.39 the cvgdiff branch fires at j = 2, with 0.38 it does not; the
difference taken from phibar_0 (0.732) would not fire at 0.39, and a sign
slip (-0.382) would fire at 0.38.
"""
import math

import numpy as np
import pytest

from oracle.aplicur import Options, RebuildRule, Trace, aplicur, ne_residual
from oracle.lsqr import STOP_BUDGET, STOP_DYNAMIC, plsqr_phase
from workloads import synth

PHIBAR_1 = 1.0
PHIBAR_2 = math.sqrt(50.0 / 131.0)


def _diag_phase(nu, sigma_l, max_iter=3):
    A = np.diag([1.0, 2.0, 3.0])
    b = np.ones(3)
    hist = []
    _, j, why = plsqr_phase(A, 0.0, b, np.zeros(3), None, nu=nu, sigma_l=sigma_l,
                            eps_lsqr=0.0, tol_ne=0.0, max_iter=max_iter, history=hist)
    return j, why, hist


def test_phibar_sequence_of_the_worked_case():
    _, _, hist = _diag_phase(math.inf, 0.0)
    assert abs(hist[0] - PHIBAR_1) <= 1e-14
    assert abs(hist[1] - PHIBAR_2) <= 1e-14
    assert hist[2] <= 1e-13


@pytest.mark.parametrize("nu,expect", [(1.1, (2, STOP_DYNAMIC)), (1.2, (3, STOP_BUDGET)),
                                       (1.14, (2, STOP_DYNAMIC)), (1.141, (3, STOP_BUDGET))])
def test_dynamic_ratio_rule_hand_worked(nu, expect):
    # ratio cvgrate_1 / cvgrate_2 = 1.140616... (module docstring)
    j, why, _ = _diag_phase(nu, 0.0)
    assert (j, why) == expect


@pytest.mark.parametrize("sigma_l,expect", [(0.39, (2, STOP_DYNAMIC)), (0.38, (3, STOP_BUDGET)),
                                            (0.3822, (2, STOP_DYNAMIC)), (0.3821, (3, STOP_BUDGET))])
def test_dynamic_cvgdiff_rule_hand_worked(sigma_l, expect):
    # cvgdiff_2 = phibar_1 - phibar_2 = 0.382198...; nu large but finite so
    # only the difference branch can fire
    j, why, _ = _diag_phase(1e9, sigma_l)
    assert (j, why) == expect


def test_dynamic_rule_is_off_in_the_final_phase():
    # nu = inf (final phase): neither branch is tested
    j, why, _ = _diag_phase(math.inf, 0.39)
    assert (j, why) == (3, STOP_BUDGET)


def test_dynamic_rule_is_not_tested_at_the_first_step():
    # a tiny nu would fire on any finite ratio, but not before j = 2
    j, why, _ = _diag_phase(1e-3, 0.0)
    assert (j, why) == (2, STOP_DYNAMIC)
    j, why, _ = _diag_phase(1e-3, 0.0, max_iter=1)
    assert (j, why) == (1, STOP_BUDGET)


# Re-preconditioning test, worked case: eps_cur = 1, nu_prec = 10.
#   step rho    gap = rho - 1   d_cur/gap           build?  d_cur after
#   1    101    100             inf                 yes     100
#   2    50     49              100/49 = 2.04       no      100
#   3    12     11              100/11 = 9.09       no      100
#   4    10.9   9.9             100/9.9 = 10.10     yes     9.9
#   5    5      4               9.9/4 = 2.475       no      9.9
#   6    1.05   0.05            9.9/0.05 = 198      yes     0.05
#   7    0.5    (final: rho <= eps_cur)             yes
# A swapped ratio (gap/d_cur, at most 0.49 here) builds only at the first and
# final steps; a sign slip (eps_cur - rho) makes every ratio negative.
REBUILD_RHOS = [101.0, 50.0, 12.0, 10.9, 5.0, 1.05, 0.5]
REBUILD_EXPECT = [True, False, False, True, False, True, True]


def test_rebuild_rule_hand_worked():
    rule = RebuildRule(eps_cur=1.0, nu_prec=10.0)
    got = [rule(r, r <= 1.0) for r in REBUILD_RHOS]
    assert got == REBUILD_EXPECT
    assert rule.d_cur == pytest.approx(-0.5)


def test_rebuild_rule_boundary():
    # d_cur/gap exactly nu_prec builds (the test is >=)
    rule = RebuildRule(eps_cur=0.0, nu_prec=4.0)
    assert rule(8.0, False)
    assert not rule(2.5, False)
    assert rule(2.0, False)


def test_single_shot_builds_only_at_the_final_step():
    rule = RebuildRule(eps_cur=1.0, nu_prec=10.0, adaptive=False)
    assert [rule(r, r <= 1.0) for r in REBUILD_RHOS] == [False] * 6 + [True]


def test_solve_trace_follows_the_rule():
    """The outer loop of the solve takes exactly the rule's decisions on the
    rho values it computes (the last step is the final one)."""
    w = synth.workload(1, 0.5)  # dense 1000 x 100, sigma_i = 10^(-6 i/100)
    tr = Trace()
    opts = Options(block=10, tol_ne=1e-10)
    aplicur(w.A, w.B, 0.0, opts, tr)
    rule = RebuildRule(eps_cur=3e-7, nu_prec=opts.nu_prec)
    n = len(tr.rhos)
    replay = [rule(r, k == n - 1) for k, r in enumerate(tr.rhos)]
    assert replay == tr.rebuild
    assert sum(tr.rebuild) >= 3 and not all(tr.rebuild)


def test_svdfree_literal_target_costs_iterations():
    """Alg. 8 takes the CUR error estimate rho as the target level.  The
    oracle floors it at eps_cur (the final build, where rho <= eps_cur, then
    uses eps_cur).  With the literal level the final P~ flattens the captured
    spectrum to rho, far below eps_cur, and ||P~|| = ||M|| / rho makes the
    certified stop (||P~|| ||A~^T r|| <= tol ||A^T b||) much stricter than
    eta needs: on the sparse sharp kappa = 1e15 set the literal level costs
    more than three times the iterations for the same tolerance."""
    A, b = synth.paper_sparse(11, 1200, 1000, "sharp15")
    res = {}
    for floor in (True, False):
        tr = Trace()
        x = aplicur(A, b, 0.0, Options(block=20, precond="svdfree", svdfree_floor=floor,
                                        max_iter=5000), tr)
        res[floor] = (tr.iters, ne_residual(A, b, x, 0.0), tr.sigma_hat[-1])
    (it_f, eta_f, t_f), (it_l, eta_l, t_l) = res[True], res[False]
    assert eta_f <= 1e-8 and eta_l <= 1e-8
    assert t_f == pytest.approx(3e-7) and t_l < 1e-8
    assert it_l > 3 * it_f, (it_f, it_l)


def test_rho_estimate_hand_worked():
    """Sec. 5.3.1: rho = 10 sqrt(2/pi) max_i ||E w_i||.  With
    E = [[3, 0, 0], [0, 4, 0]], w_1 = (1, 1, 0), w_2 = (0, 0, 1):
    ||E w_1|| = ||(3, 4)|| = 5, ||E w_2|| = 0, so rho = 50 sqrt(2/pi)
    = 39.894228040143...."""
    from oracle.cur import rho_estimate
    E = np.array([[3.0, 0.0, 0.0], [0.0, 4.0, 0.0]])
    W = np.array([[1.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    assert rho_estimate(E, W) == pytest.approx(39.894228040143, rel=1e-12)
