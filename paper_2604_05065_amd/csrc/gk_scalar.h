// LSQR scalar recurrences (Sec. 2.2, stopping tests of Sec. 5.3.2) on one
// FP64 state copy, shared by the single-column and the blocked kernels.
#pragma once

#include "common.h"

namespace aplicur {

// Modes of the forward kernels: PLAIN finishes alpha from the backward
// kernel's partials (slot 1 -> slot 0) and applies the y/w update; PRE reads
// slot 0 (alpha finished by the P^{-1} kernel); MATVEC uses slot 0 as given
// (alpha = beta = 1).
enum FwdMode { kFwdPlain = 0, kFwdPre = 1, kFwdMatvec = 2 };

// ---------------------------------------------------------------- scalar update
// One LSQR scalar step on a state copy: the initial step (alpha_1, beta_1) or
// the Givens rotation of the previous iteration with the new alpha.
__device__ inline void scalar_step(GKState& s, double alpha) {
  if (!(alpha == alpha) || isinf(alpha)) {
    s.stop = 1;
    s.reason = 6;
    s.pending = 0;
    return;
  }
  if (s.init) {
    s.init = 0;
    const double beta = s.beta;
    s.alpha = alpha;
    s.rhobar = alpha;
    s.phibar = beta;
    s.beta1 = beta;
    s.h2 = (alpha * beta) * (alpha * beta);
    s.anorm2 = alpha * alpha;
    s.phibar_prev = beta;
    s.have_rate1 = 0;
    s.iter = 0;
    s.coef_y = 0.0;
    s.coef_w = 0.0;
    s.pending = 1;  // w = v / alpha
    s.arnorm = alpha * beta;
    if (alpha == 0.0 || beta == 0.0) {
      s.stop = 1;
      s.reason = kStopExact;
      s.pending = 0;
    } else if (s.max_iter <= 0) {
      s.stop = 1;
      s.reason = kStopBudget;
      s.pending = 0;
    }
    return;
  }
  const double beta = s.beta;
  s.alpha = alpha;
  s.anorm2 += alpha * alpha + beta * beta;
  const double rho = hypot(s.rhobar, beta);
  const double c = s.rhobar / rho, sn = beta / rho;
  const double theta = sn * alpha;
  s.rhobar = -c * alpha;
  const double phi = c * s.phibar;
  const double phibar = sn * s.phibar;
  s.phibar = phibar;
  s.coef_y = phi / rho;
  s.coef_w = theta / rho;
  s.pending = 1;
  s.iter += 1;
  const double arnorm = phibar * alpha * fabs(c);
  s.arnorm = arnorm;
  int reason = kStopNone;
  if (beta == 0.0 || alpha == 0.0) {
    reason = kStopExact;
  } else if (s.pnorm * arnorm <= s.tol_abs || arnorm <= s.rel_tol * sqrt(s.h2)) {
    reason = kStopMetric;
  } else if (s.eps_lsqr > 0.0 && (arnorm <= s.eps_lsqr * sqrt(s.anorm2) * phibar || phibar <= s.baug_eps)) {
    reason = kStopLsqr;
  } else {
    const double rate = phibar > 0.0 ? log(s.phibar_prev / phibar) : INFINITY;
    if (!s.have_rate1) {
      s.rate1 = rate;
      s.have_rate1 = 1;
    } else if (!isinf(s.nu)) {
      const double ratio = rate <= 0.0 ? INFINITY : s.rate1 / rate;
      if (ratio > s.nu || (s.phibar_prev - phibar) < s.sigma_l) reason = kStopDynamic;
    }
    if (reason == kStopNone) s.phibar_prev = phibar;
  }
  if (reason == kStopNone && s.iter >= s.max_iter) reason = kStopBudget;
  if (reason != kStopNone) {
    s.stop = 1;
    s.reason = reason;
  }
}

// beta = sqrt(sum of squares); flags non-finite values and a zero residual
// at the phase start (nothing to do).
__device__ __forceinline__ void beta_step(GKState& s, double b2) {
  const double b = sqrt(b2);
  s.beta = b;
  if (!(b == b) || isinf(b)) {
    s.stop = 1;
    s.reason = 6;
  } else if (b == 0.0 && s.init) {
    s.beta1 = 0.0;
    s.stop = 1;
    s.reason = kStopExact;
  }
}

}  // namespace aplicur
