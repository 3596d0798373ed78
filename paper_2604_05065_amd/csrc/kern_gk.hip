// Golub-Kahan bidiagonalisation with the LSQR Givens recurrences (Sec. 2.2)
// on the augmented, right-preconditioned operator  A~ = A_mu P^{-1},
// A_mu = [A; delta I]  (delta = sqrt(mu)), one iteration being
//
//     beta u  = A~ v   - alpha u      (forward kernel; P^{-1} v first if P != I)
//     alpha v = A~^T u - beta  v      (backward kernel; then P^{-T})
//     Givens rotation, y += (phi/rho) w, w = v - (theta/rho) w.
//
// Reductions without fences: a kernel that produces a norm writes one
// partial sum per workgroup; every workgroup of the next (consuming) kernel
// sums those partials itself in a fixed order, so all workgroups hold the
// bitwise-identical scalar and take identical decisions.  The FP64 scalar
// state lives in two slots: slot 0 is written by the kernel that finishes
// alpha (forward kernel, or the P^{-1} kernel with a preconditioner), slot 1
// by the backward kernel that finishes beta; a kernel never reads the slot
// it writes.  Normalisation by 1/beta and 1/alpha is folded into the next
// consumer; the Givens update of iteration j and the y/w update are done by
// the first kernel of iteration j + 1, which also evaluates the stopping
// tests of Sec. 5.3.2 and, on stopping, applies the last y update itself.
#include "kernels.h"

namespace aplicur {

constexpr int kMaxGrid = 1024;

// ---------------------------------------------------------------- scalar update
// One LSQR scalar step on a state copy: the initial step (alpha_1, beta_1) or
// the Givens rotation of the previous iteration with the new alpha.
__device__ void scalar_step(GKState& s, double alpha) {
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
  } else if (s.pnorm * arnorm <= s.tol_abs) {
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

__device__ __forceinline__ bool stopped(const GKState* st) { return st[0].stop || st[1].stop; }

// Load slot `in` into LDS; when `alpha_part` is given, finish alpha from the
// partials and take the scalar step; workgroup 0 stores the result in `out`.
__device__ __forceinline__ void load_and_step(GKState& s, const GKState* in, GKState* out,
                                              const double* alpha_part, int alpha_count) {
  if (threadIdx.x == 0) s = *in;
  __syncthreads();
  if (alpha_part) {
    const double a2 = reduce_all(alpha_part, alpha_count);
    if (threadIdx.x == 0) scalar_step(s, sqrt(a2));
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) *out = s;
  }
}

// ---------------------------------------------------------------- CSR row dot
template <class TA, class V, class X>
__device__ __forceinline__ V csr_dot(const int* __restrict__ rp, const int* __restrict__ ci,
                                     const TA* __restrict__ val, const X* __restrict__ x, long long row,
                                     int lane, int G) {
  V acc = 0;
  const int b = rp[row], e = rp[row + 1];
  for (int k = b + lane; k < e; k += G) acc += (V)val[k] * (V)x[ci[k]];
  for (int off = G >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
  return acc;
}

// Forward modes: GK_PLAIN finishes alpha and takes the scalar step (no
// preconditioner); GK_PRE reads alpha from slot 0 (finished by the P^{-1}
// kernel); MATVEC uses the state as given (alpha = beta = 1, delta = 0).
enum FwdMode { kFwdPlain = 0, kFwdPre = 1, kFwdMatvec = 2 };

// Bottom (n-length) part of the forward kernel: u_bot update and the y/w
// update of the previous iteration (or, on stopping, the last y update).
template <class V>
__device__ __forceinline__ double fwd_bottom(long long j, const V* tin, V* u_bot, const V* v, V* w, V* y,
                                             const GKState& s, V ts, V cu, bool do_pending) {
  double sq = 0.0;
  if (s.delta > 0.0) {
    const V ub = (V)s.delta * (tin[j] * ts) - cu * u_bot[j];
    u_bot[j] = ub;
    sq = (double)ub * (double)ub;
  }
  if (do_pending && s.pending) {
    const V vj = v[j] * ts;
    const V wj = w[j];
    y[j] += (V)s.coef_y * wj;
    w[j] = vj - (V)s.coef_w * wj;
  }
  return sq;
}

template <class V>
__device__ __forceinline__ void final_y_update(long long n, V* y, const V* w, const GKState& s, int first_block,
                                               int nblocks) {
  if (!s.pending) return;
  for (long long j = (long long)(blockIdx.x - first_block) * kBlock + threadIdx.x; j < n;
       j += (long long)nblocks * kBlock)
    y[j] += (V)s.coef_y * w[j];
}

// u_top <- A (tin / alpha) - (alpha / beta) u_top ; u_bot <- delta tin/alpha - (alpha/beta) u_bot
template <class TA, class V, int MODE>
__global__ void __launch_bounds__(kBlock)
    k_fwd_csr(const int* __restrict__ rp, const int* __restrict__ ci, const TA* __restrict__ val, long long m,
              long long n, const V* tin, V* u_top, V* u_bot, const V* v, V* w, V* y, GKState* st,
              const double* alpha_part, int alpha_count, double* beta_part, int G, int row_blocks) {
  __shared__ GKState s;
  if (MODE != kFwdMatvec && stopped(st)) return;
  load_and_step(s, MODE == kFwdPlain ? &st[1] : &st[0], &st[0], MODE == kFwdPlain ? alpha_part : nullptr,
                alpha_count);
  const bool bottom = (int)blockIdx.x >= row_blocks;
  const int nb = gridDim.x - row_blocks;
  if (MODE == kFwdPlain && s.stop) {
    if (bottom) final_y_update<V>(n, y, w, s, row_blocks, nb);
    return;
  }
  const V ts = (V)(1.0 / s.alpha), cu = (V)(s.alpha / s.beta);
  double sq = 0.0;
  if (!bottom) {
    const int rpb = kBlock / G, lane = threadIdx.x % G;
    for (long long row = (long long)blockIdx.x * rpb + threadIdx.x / G; row < m; row += (long long)row_blocks * rpb) {
      const V dot = csr_dot<TA, V>(rp, ci, val, tin, row, lane, G);
      if (lane == 0) {
        const V un = dot * ts - cu * u_top[row];
        u_top[row] = un;
        sq += (double)un * (double)un;
      }
    }
  } else {
    for (long long j = (long long)(blockIdx.x - row_blocks) * kBlock + threadIdx.x; j < n; j += (long long)nb * kBlock)
      sq += fwd_bottom<V>(j, tin, u_bot, v, w, y, s, ts, cu, MODE == kFwdPlain);
  }
  const double bs = block_sum(sq);
  if (threadIdx.x == 0) beta_part[blockIdx.x] = bs;
}

// Dense row-major A: one wave per row.
template <class TA, class V, int MODE>
__global__ void __launch_bounds__(kBlock)
    k_fwd_dense(const TA* __restrict__ A, long long m, long long n, long long ld, const V* tin, V* u_top,
                V* u_bot, const V* v, V* w, V* y, GKState* st, const double* alpha_part, int alpha_count,
                double* beta_part, int row_blocks) {
  __shared__ GKState s;
  if (MODE != kFwdMatvec && stopped(st)) return;
  load_and_step(s, MODE == kFwdPlain ? &st[1] : &st[0], &st[0], MODE == kFwdPlain ? alpha_part : nullptr,
                alpha_count);
  const bool bottom = (int)blockIdx.x >= row_blocks;
  const int nb = gridDim.x - row_blocks;
  if (MODE == kFwdPlain && s.stop) {
    if (bottom) final_y_update<V>(n, y, w, s, row_blocks, nb);
    return;
  }
  const V ts = (V)(1.0 / s.alpha), cu = (V)(s.alpha / s.beta);
  double sq = 0.0;
  if (!bottom) {
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    constexpr int rpb = kBlock / kWave;
    for (long long row = (long long)blockIdx.x * rpb + wv; row < m; row += (long long)row_blocks * rpb) {
      const TA* a = A + row * ld;
      V acc = 0;
      for (long long c = lane; c < n; c += kWave) acc += (V)a[c] * tin[c];
      acc = wave_sum(acc);
      if (lane == 0) {
        const V un = acc * ts - cu * u_top[row];
        u_top[row] = un;
        sq += (double)un * (double)un;
      }
    }
  } else {
    for (long long j = (long long)(blockIdx.x - row_blocks) * kBlock + threadIdx.x; j < n; j += (long long)nb * kBlock)
      sq += fwd_bottom<V>(j, tin, u_bot, v, w, y, s, ts, cu, MODE == kFwdPlain);
  }
  const double bs = block_sum(sq);
  if (threadIdx.x == 0) beta_part[blockIdx.x] = bs;
}

// Backward: beta from the forward partials (or the state when beta_part is
// null), g = (A^T u_top + delta u_bot) / beta.  PLAIN: v_raw <- g -
// (beta/alpha) v_raw (g at the phase start); otherwise g is stored for
// P^{-T}.  Partials of the produced vector's squared norm go to alpha_part.
template <class V, bool PLAIN>
__device__ __forceinline__ double bwd_epilogue(long long j, V dot, const V* u_bot, V* v, V* g, const GKState& s,
                                               V ib, V cv) {
  V gj = dot * ib;
  if (s.delta > 0.0) gj += (V)s.delta * u_bot[j] * ib;
  if (PLAIN) {
    const V vn = s.init ? gj : gj - cv * v[j];
    v[j] = vn;
    return (double)vn * (double)vn;
  } else {
    g[j] = gj;
    return (double)gj * (double)gj;
  }
}

// Returns false when the kernel must not do its work (stopped / beta == 0).
__device__ __forceinline__ bool bwd_prologue(GKState& s, GKState* st, const double* beta_part, int beta_count,
                                             double* alpha_part) {
  if (threadIdx.x == 0) s = st[0];
  __syncthreads();
  if (beta_part) {
    const double b2 = reduce_all(beta_part, beta_count);
    if (threadIdx.x == 0) {
      const double b = sqrt(b2);
      s.beta = b;
      if (!(b == b) || isinf(b)) {
        s.stop = 1;
        s.reason = 6;
      } else if (b == 0.0 && s.init) {
        s.stop = 1;  // zero residual at the phase start: nothing to do
        s.reason = kStopExact;
      }
    }
    __syncthreads();
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) st[1] = s;
  if (s.stop) return false;
  if (s.beta == 0.0) {  // exact solution reached: alpha = 0 ends the phase in the next kernel
    if (threadIdx.x == 0) alpha_part[blockIdx.x] = 0.0;
    return false;
  }
  return true;
}

template <class TA, class V, bool PLAIN>
__global__ void __launch_bounds__(kBlock)
    k_bwd_csr(const int* __restrict__ tp, const int* __restrict__ ti, const TA* __restrict__ tv, long long n,
              const V* u_top, const V* u_bot, V* v, V* g, GKState* st, const double* beta_part, int beta_count,
              double* alpha_part, int G) {
  __shared__ GKState s;
  if (stopped(st)) return;
  if (!bwd_prologue(s, st, beta_part, beta_count, alpha_part)) return;
  const V ib = (V)(1.0 / s.beta), cv = (V)(s.beta / s.alpha);
  double sq = 0.0;
  const int rpb = kBlock / G, lane = threadIdx.x % G;
  for (long long j = (long long)blockIdx.x * rpb + threadIdx.x / G; j < n; j += (long long)gridDim.x * rpb) {
    const V dot = csr_dot<TA, V>(tp, ti, tv, u_top, j, lane, G);
    if (lane == 0) sq += bwd_epilogue<V, PLAIN>(j, dot, u_bot, v, g, s, ib, cv);
  }
  const double bs = block_sum(sq);
  if (threadIdx.x == 0) alpha_part[blockIdx.x] = bs;
}

// Dense A^T u: partial sums over row chunks (threads along columns, coalesced).
template <class TA, class V>
__global__ void __launch_bounds__(kBlock)
    k_bwd_dense_part(const TA* __restrict__ A, long long m, long long n, long long ld, const V* __restrict__ u_top,
                     double* part, long long rpc, const GKState* st) {
  if (st && stopped(st)) return;
  const long long j = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (j >= n) return;
  const long long i0 = (long long)blockIdx.y * rpc;
  const long long i1 = min(m, i0 + rpc);
  V acc = 0;
  for (long long i = i0; i < i1; ++i) acc += (V)A[i * ld + j] * u_top[i];
  part[(long long)blockIdx.y * n + j] = (double)acc;
}

template <class V, bool PLAIN>
__global__ void __launch_bounds__(kBlock)
    k_bwd_dense_red(const double* __restrict__ part, int chunks, long long n, const V* u_bot, V* v, V* g,
                    GKState* st, const double* beta_part, int beta_count, double* alpha_part) {
  __shared__ GKState s;
  if (stopped(st)) return;
  if (!bwd_prologue(s, st, beta_part, beta_count, alpha_part)) return;
  const V ib = (V)(1.0 / s.beta), cv = (V)(s.beta / s.alpha);
  double sq = 0.0;
  for (long long j = (long long)blockIdx.x * kBlock + threadIdx.x; j < n; j += (long long)gridDim.x * kBlock) {
    double acc = 0.0;
    for (int c = 0; c < chunks; ++c) acc += part[(long long)c * n + j];
    sq += bwd_epilogue<V, PLAIN>(j, (V)acc, u_bot, v, g, s, ib, cv);
  }
  const double bs = block_sum(sq);
  if (threadIdx.x == 0) alpha_part[blockIdx.x] = bs;
}

// ---------------------------------------------------------------- explicit P apply
// c = d .* (V^T z): chunk partials (threads along the ell columns of the
// row-major V), then an ordered sum over chunks.
template <class V>
__global__ void __launch_bounds__(kBlock)
    k_pa_part(const double* __restrict__ Vh, long long n, int ell, long long ldv, const V* __restrict__ z,
              double* part, long long rpc, const GKState* st) {
  if (st && stopped(st)) return;
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= ell) return;
  const long long i0 = (long long)blockIdx.y * rpc;
  const long long i1 = min(n, i0 + rpc);
  double acc = 0.0;
  for (long long i = i0; i < i1; ++i) acc += Vh[i * ldv + k] * (double)z[i];
  part[(long long)blockIdx.y * ell + k] = acc;
}

__global__ void k_pa_red(const double* __restrict__ part, int chunks, int ell, const double* __restrict__ d,
                         double* c, const GKState* st) {
  if (st && stopped(st)) return;
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= ell) return;
  double acc = 0.0;
  for (int ch = 0; ch < chunks; ++ch) acc += part[(long long)ch * ell + k];
  c[k] = d[k] * acc;
}

__device__ __forceinline__ double vrow_dot(const double* __restrict__ Vh, long long ldv, int ell,
                                           const double* __restrict__ c, long long i, int lane) {
  double acc = 0.0;
  const double* r = Vh + i * ldv;
  for (int k = lane; k < ell; k += kWave) acc += r[k] * c[k];
  return wave_sum(acc);
}

// First kernel of a preconditioned iteration: finishes alpha (partials of
// the previous P^{-T} kernel), takes the scalar step, applies the y/w update,
// and forms t = v_raw + V c (= P^{-1} v_raw).
template <class V>
__global__ void __launch_bounds__(kBlock)
    k_pa_fwd(const double* __restrict__ Vh, long long n, int ell, long long ldv, const double* __restrict__ c,
             const V* v, V* t, V* w, V* y, GKState* st, const double* alpha_part, int alpha_count) {
  __shared__ GKState s;
  if (stopped(st)) return;
  load_and_step(s, &st[1], &st[0], alpha_part, alpha_count);
  if (s.stop) {
    final_y_update<V>(n, y, w, s, 0, gridDim.x);
    return;
  }
  const double ia = 1.0 / s.alpha;
  const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  constexpr int rpb = kBlock / kWave;
  for (long long i = (long long)blockIdx.x * rpb + wv; i < n; i += (long long)gridDim.x * rpb) {
    const double dot = vrow_dot(Vh, ldv, ell, c, i, lane);
    if (lane == 0) {
      const V vi = v[i];
      t[i] = (V)((double)vi + dot);
      if (s.pending) {
        const V wi = w[i];
        y[i] += (V)s.coef_y * wi;
        w[i] = (V)((double)vi * ia) - (V)s.coef_w * wi;
      }
    }
  }
}

// v_raw <- (g + V c) - (beta/alpha) v_raw  (g + V c at the phase start);
// partials of ||v_raw||^2 for the next iteration's alpha.
template <class V>
__global__ void __launch_bounds__(kBlock)
    k_pa_bwd(const double* __restrict__ Vh, long long n, int ell, long long ldv, const double* __restrict__ c,
             const V* g, V* v, const GKState* st, double* alpha_part) {
  if (stopped(st)) return;
  const GKState& s = st[1];
  const int init = s.init;
  const double cv = s.beta / s.alpha;
  const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  constexpr int rpb = kBlock / kWave;
  double sq = 0.0;
  for (long long i = (long long)blockIdx.x * rpb + wv; i < n; i += (long long)gridDim.x * rpb) {
    const double dot = vrow_dot(Vh, ldv, ell, c, i, lane);
    if (lane == 0) {
      const double pg = (double)g[i] + dot;
      const V vn = init ? (V)pg : (V)(pg - cv * (double)v[i]);
      v[i] = vn;
      sq += (double)vn * (double)vn;
    }
  }
  const double bs = block_sum(sq);
  if (threadIdx.x == 0) alpha_part[blockIdx.x] = bs;
}

// x += y + V c  (x in FP64).
template <class V>
__global__ void __launch_bounds__(kBlock)
    k_pa_x(const double* __restrict__ Vh, long long n, int ell, long long ldv, const double* __restrict__ c,
           const V* y, double* x) {
  const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  constexpr int rpb = kBlock / kWave;
  for (long long i = (long long)blockIdx.x * rpb + wv; i < n; i += (long long)gridDim.x * rpb) {
    const double dot = vrow_dot(Vh, ldv, ell, c, i, lane);
    if (lane == 0) x[i] += (double)y[i] + dot;
  }
}

// ---------------------------------------------------------------- phase start / helpers
// r_top = b - A x (FP64, values widened), r_bot = bot_scale b_bot - delta x;
// partials of ||r||^2 into beta_part.
template <class TA>
__global__ void __launch_bounds__(kBlock)
    k_resid_csr(const int* __restrict__ rp, const int* __restrict__ ci, const TA* __restrict__ val, long long m,
                long long n, const double* __restrict__ b, const double* b_bot, double bot_scale, const double* x,
                int x_zero, double* r_top, double* r_bot, const GKState* st, double* beta_part, int G,
                int row_blocks) {
  const double delta = st[0].delta;
  double sq = 0.0;
  if ((int)blockIdx.x < row_blocks) {
    const int rpb = kBlock / G, lane = threadIdx.x % G;
    for (long long row = (long long)blockIdx.x * rpb + threadIdx.x / G; row < m; row += (long long)row_blocks * rpb) {
      const double dot = x_zero ? 0.0 : csr_dot<TA, double>(rp, ci, val, x, row, lane, G);
      if (lane == 0) {
        const double r = (b ? b[row] : 0.0) - dot;
        r_top[row] = r;
        sq += r * r;
      }
    }
  } else if (delta > 0.0) {
    const int nb = gridDim.x - row_blocks;
    for (long long j = (long long)(blockIdx.x - row_blocks) * kBlock + threadIdx.x; j < n; j += (long long)nb * kBlock) {
      double r = x_zero ? 0.0 : -delta * x[j];
      if (b_bot) r += bot_scale * b_bot[j];
      r_bot[j] = r;
      sq += r * r;
    }
  }
  const double bs = block_sum(sq);
  if (threadIdx.x == 0) beta_part[blockIdx.x] = bs;
}

template <class TA>
__global__ void __launch_bounds__(kBlock)
    k_resid_dense(const TA* __restrict__ A, long long m, long long n, long long ld, const double* __restrict__ b,
                  const double* b_bot, double bot_scale, const double* x, int x_zero, double* r_top, double* r_bot,
                  const GKState* st, double* beta_part, int row_blocks) {
  const double delta = st[0].delta;
  double sq = 0.0;
  if ((int)blockIdx.x < row_blocks) {
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    constexpr int rpb = kBlock / kWave;
    for (long long row = (long long)blockIdx.x * rpb + wv; row < m; row += (long long)row_blocks * rpb) {
      double acc = 0.0;
      if (!x_zero) {
        const TA* a = A + row * ld;
        for (long long c = lane; c < n; c += kWave) acc += (double)a[c] * x[c];
        acc = wave_sum(acc);
      }
      if (lane == 0) {
        const double r = (b ? b[row] : 0.0) - acc;
        r_top[row] = r;
        sq += r * r;
      }
    }
  } else if (delta > 0.0) {
    const int nb = gridDim.x - row_blocks;
    for (long long j = (long long)(blockIdx.x - row_blocks) * kBlock + threadIdx.x; j < n; j += (long long)nb * kBlock) {
      double r = x_zero ? 0.0 : -delta * x[j];
      if (b_bot) r += bot_scale * b_bot[j];
      r_bot[j] = r;
      sq += r * r;
    }
  }
  const double bs = block_sum(sq);
  if (threadIdx.x == 0) beta_part[blockIdx.x] = bs;
}

// One workgroup: finish a reduction into the state.  mode 0: alpha and the
// scalar step (slot 1 -> slot 0); mode 1: beta1 = sqrt(sum) in slot 0.
__global__ void __launch_bounds__(kBlock) k_consume(GKState* st, const double* part, int count, int mode) {
  __shared__ GKState s;
  const double tot = reduce_all(part, count);
  if (threadIdx.x == 0) {
    s = mode == 0 ? st[1] : st[0];
    if (mode == 0) {
      if (!s.stop) scalar_step(s, sqrt(tot));
    } else {
      s.beta1 = sqrt(tot);
    }
    st[0] = s;
  }
}

template <class V>
__global__ void k_axpy_x(long long n, const V* y, double* x) {
  for (long long j = (long long)blockIdx.x * kBlock + threadIdx.x; j < n; j += (long long)gridDim.x * kBlock)
    x[j] += (double)y[j];
}

template <class V>
__global__ void k_fill_zero(V* p, long long n) {
  for (long long j = (long long)blockIdx.x * kBlock + threadIdx.x; j < n; j += (long long)gridDim.x * kBlock) p[j] = (V)0;
}

template <class V>
void fill_zero(V* p, long long n, hipStream_t s) {
  if (n <= 0) return;
  unsigned g = ceil_div(n, kBlock);
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_fill_zero<V>, dim3(g), dim3(kBlock), 0, s, p, n);
}
template void fill_zero<double>(double*, long long, hipStream_t);
template void fill_zero<float>(float*, long long, hipStream_t);

// ---------------------------------------------------------------- host launchers
static unsigned clamp_grid(long long want) {
  if (want < 1) return 1;
  return (unsigned)(want > kMaxGrid ? kMaxGrid : want);
}
static unsigned nbottom(long long n) {
  long long b = (n + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  return (unsigned)(b > 256 ? 256 : b);
}
static unsigned fwd_row_blocks(const OpDesc& A) {
  if (A.csr) {
    const int rpb = kBlock / A.group;
    return clamp_grid((A.m + rpb - 1) / rpb);
  }
  return clamp_grid((A.m + 3) / 4);
}
static unsigned fwd_grid(const OpDesc& A) { return fwd_row_blocks(A) + nbottom(A.n); }
static unsigned bwd_grid(const OpDesc& A) {
  if (A.csr) {
    const int rpb = kBlock / A.t_group;
    return clamp_grid((A.n + rpb - 1) / rpb);
  }
  return clamp_grid(ceil_div(A.n, kBlock));
}
static unsigned rows_grid(long long n) { return clamp_grid((n + 3) / 4); }

template <class V, int MODE>
static void launch_fwd(const OpDesc& A, const V* tin, GKVecs<V> vec, GKState* st, GKWork& wk, hipStream_t s) {
  const unsigned rb = fwd_row_blocks(A);
  const unsigned grid = rb + nbottom(A.n);
  const int ac = (int)wk.alpha_count;
  if (A.csr) {
    if (A.f64)
      hipLaunchKernelGGL((k_fwd_csr<double, V, MODE>), dim3(grid), dim3(kBlock), 0, s, A.row_ptr, A.col_idx,
                         (const double*)A.val, A.m, A.n, tin, vec.u_top, vec.u_bot, vec.v, vec.w, vec.y, st,
                         wk.alpha_part, ac, wk.beta_part, A.group, (int)rb);
    else
      hipLaunchKernelGGL((k_fwd_csr<float, V, MODE>), dim3(grid), dim3(kBlock), 0, s, A.row_ptr, A.col_idx,
                         (const float*)A.val, A.m, A.n, tin, vec.u_top, vec.u_bot, vec.v, vec.w, vec.y, st,
                         wk.alpha_part, ac, wk.beta_part, A.group, (int)rb);
  } else {
    if (A.f64)
      hipLaunchKernelGGL((k_fwd_dense<double, V, MODE>), dim3(grid), dim3(kBlock), 0, s, (const double*)A.val, A.m,
                         A.n, A.ld, tin, vec.u_top, vec.u_bot, vec.v, vec.w, vec.y, st, wk.alpha_part, ac,
                         wk.beta_part, (int)rb);
    else
      hipLaunchKernelGGL((k_fwd_dense<float, V, MODE>), dim3(grid), dim3(kBlock), 0, s, (const float*)A.val, A.m,
                         A.n, A.ld, tin, vec.u_top, vec.u_bot, vec.v, vec.w, vec.y, st, wk.alpha_part, ac,
                         wk.beta_part, (int)rb);
  }
  wk.beta_count = grid;
}

// beta_from_part: finish beta from wk.beta_part (else the state's beta is used).
template <class V, bool PLAIN>
static void launch_bwd(const OpDesc& A, const V* u_top, const V* u_bot, V* v, V* g, GKState* st, GKWork& wk,
                       bool beta_from_part, hipStream_t s) {
  const double* bp = beta_from_part ? wk.beta_part : nullptr;
  const int bc = (int)wk.beta_count;
  if (A.csr) {
    const unsigned grid = bwd_grid(A);
    if (A.f64)
      hipLaunchKernelGGL((k_bwd_csr<double, V, PLAIN>), dim3(grid), dim3(kBlock), 0, s, A.t_ptr, A.t_idx,
                         (const double*)A.t_val, A.n, u_top, u_bot, v, g, st, bp, bc, wk.alpha_part, A.t_group);
    else
      hipLaunchKernelGGL((k_bwd_csr<float, V, PLAIN>), dim3(grid), dim3(kBlock), 0, s, A.t_ptr, A.t_idx,
                         (const float*)A.t_val, A.n, u_top, u_bot, v, g, st, bp, bc, wk.alpha_part, A.t_group);
    wk.alpha_count = grid;
  } else {
    const long long rpc = (A.m + A.chunks - 1) / A.chunks;
    dim3 g1(ceil_div(A.n, kBlock), A.chunks);
    if (A.f64)
      hipLaunchKernelGGL((k_bwd_dense_part<double, V>), g1, dim3(kBlock), 0, s, (const double*)A.val, A.m, A.n, A.ld,
                         u_top, A.part, rpc, (const GKState*)st);
    else
      hipLaunchKernelGGL((k_bwd_dense_part<float, V>), g1, dim3(kBlock), 0, s, (const float*)A.val, A.m, A.n, A.ld,
                         u_top, A.part, rpc, (const GKState*)st);
    const unsigned grid = bwd_grid(A);
    hipLaunchKernelGGL((k_bwd_dense_red<V, PLAIN>), dim3(grid), dim3(kBlock), 0, s, A.part, A.chunks, A.n, u_bot, v,
                       g, st, bp, bc, wk.alpha_part);
    wk.alpha_count = grid;
  }
}

template <class V>
static void launch_pa_c(const PrecDesc& P, long long n, const V* z, const GKState* st, hipStream_t s) {
  const long long rpc = (n + P.chunks - 1) / P.chunks;
  hipLaunchKernelGGL((k_pa_part<V>), dim3(ceil_div(P.ell, kBlock), P.chunks), dim3(kBlock), 0, s, P.V, n, P.ell,
                     P.ldv, z, P.part, rpc, st);
  hipLaunchKernelGGL(k_pa_red, dim3(ceil_div(P.ell, kBlock)), dim3(kBlock), 0, s, P.part, P.chunks, P.ell, P.d, P.c,
                     st);
}

template <class V>
void gk_iteration(const OpDesc& A, const PrecDesc* P, GKVecs<V> vec, GKState* st, GKWork& wk, hipStream_t s) {
  if (!P) {
    launch_fwd<V, kFwdPlain>(A, vec.v, vec, st, wk, s);
    launch_bwd<V, true>(A, vec.u_top, vec.u_bot, vec.v, vec.g, st, wk, true, s);
    return;
  }
  launch_pa_c<V>(*P, A.n, vec.v, st, s);
  const unsigned rg = rows_grid(A.n);
  hipLaunchKernelGGL((k_pa_fwd<V>), dim3(rg), dim3(kBlock), 0, s, P->V, A.n, P->ell, P->ldv, P->c, vec.v, vec.t,
                     vec.w, vec.y, st, wk.alpha_part, (int)wk.alpha_count);
  launch_fwd<V, kFwdPre>(A, vec.t, vec, st, wk, s);
  launch_bwd<V, false>(A, vec.u_top, vec.u_bot, vec.v, vec.g, st, wk, true, s);
  launch_pa_c<V>(*P, A.n, vec.g, st, s);
  hipLaunchKernelGGL((k_pa_bwd<V>), dim3(rg), dim3(kBlock), 0, s, P->V, A.n, P->ell, P->ldv, P->c, vec.g, vec.v,
                     (const GKState*)st, wk.alpha_part);
  wk.alpha_count = rg;
}

static void launch_resid(const OpDesc& A, const double* b, const double* b_bot, double bot_scale, const double* x,
                         double* r_top, double* r_bot, GKState* st, GKWork& wk, hipStream_t s) {
  const int x_zero = (x == nullptr);
  const unsigned rb = fwd_row_blocks(A);
  const unsigned grid = rb + nbottom(A.n);
  if (A.csr) {
    if (A.f64)
      hipLaunchKernelGGL((k_resid_csr<double>), dim3(grid), dim3(kBlock), 0, s, A.row_ptr, A.col_idx,
                         (const double*)A.val, A.m, A.n, b, b_bot, bot_scale, x, x_zero, r_top, r_bot,
                         (const GKState*)st, wk.beta_part, A.group, (int)rb);
    else
      hipLaunchKernelGGL((k_resid_csr<float>), dim3(grid), dim3(kBlock), 0, s, A.row_ptr, A.col_idx,
                         (const float*)A.val, A.m, A.n, b, b_bot, bot_scale, x, x_zero, r_top, r_bot,
                         (const GKState*)st, wk.beta_part, A.group, (int)rb);
  } else {
    if (A.f64)
      hipLaunchKernelGGL((k_resid_dense<double>), dim3(grid), dim3(kBlock), 0, s, (const double*)A.val, A.m, A.n,
                         A.ld, b, b_bot, bot_scale, x, x_zero, r_top, r_bot, (const GKState*)st, wk.beta_part,
                         (int)rb);
    else
      hipLaunchKernelGGL((k_resid_dense<float>), dim3(grid), dim3(kBlock), 0, s, (const float*)A.val, A.m, A.n,
                         A.ld, b, b_bot, bot_scale, x, x_zero, r_top, r_bot, (const GKState*)st, wk.beta_part,
                         (int)rb);
  }
  wk.beta_count = grid;
}

template <class V>
void gk_phase_init(const OpDesc& A, const PrecDesc* P, const double* b, const double* b_bot, double bot_scale,
                   const double* x, GKVecs<V> vec, double* r_top64, double* r_bot64, GKState* st, GKWork& wk,
                   hipStream_t s) {
  static_assert(sizeof(V) == 8, "only the FP64 vector path is implemented here");
  launch_resid(A, b, b_bot, bot_scale, x, r_top64, r_bot64, st, wk, s);
  fill_zero<V>(vec.y, A.n, s);
  fill_zero<V>(vec.w, A.n, s);
  if (!P) {
    launch_bwd<V, true>(A, (const V*)r_top64, (const V*)r_bot64, vec.v, vec.g, st, wk, true, s);
  } else {
    launch_bwd<V, false>(A, (const V*)r_top64, (const V*)r_bot64, vec.v, vec.g, st, wk, true, s);
    launch_pa_c<V>(*P, A.n, vec.g, st, s);
    const unsigned rg = rows_grid(A.n);
    hipLaunchKernelGGL((k_pa_bwd<V>), dim3(rg), dim3(kBlock), 0, s, P->V, A.n, P->ell, P->ldv, P->c, vec.g, vec.v,
                       (const GKState*)st, wk.alpha_part);
    wk.alpha_count = rg;
  }
}

template <class V>
void gk_phase_finish(const OpDesc& A, const PrecDesc* P, GKVecs<V> vec, double* x, GKState* st, hipStream_t s) {
  (void)st;
  const unsigned g = clamp_grid(ceil_div(A.n, kBlock));
  if (!P) {
    hipLaunchKernelGGL((k_axpy_x<V>), dim3(g), dim3(kBlock), 0, s, A.n, vec.y, x);
  } else {
    launch_pa_c<V>(*P, A.n, vec.y, nullptr, s);
    hipLaunchKernelGGL((k_pa_x<V>), dim3(rows_grid(A.n)), dim3(kBlock), 0, s, P->V, A.n, P->ell, P->ldv, P->c, vec.y,
                       x);
  }
}

template void gk_iteration<double>(const OpDesc&, const PrecDesc*, GKVecs<double>, GKState*, GKWork&, hipStream_t);
template void gk_phase_init<double>(const OpDesc&, const PrecDesc*, const double*, const double*, double,
                                    const double*, GKVecs<double>, double*, double*, GKState*, GKWork&, hipStream_t);
template void gk_phase_finish<double>(const OpDesc&, const PrecDesc*, GKVecs<double>, double*, GKState*,
                                      hipStream_t);

// eta support: ||A_mu^T r|| for r = [b - A x; -delta x] into st[0].h2 (and
// ||r|| into st[0].beta1), through the plain phase-start kernels.
void gk_normal_residual(const OpDesc& A, const double* b, const double* b_bot, double bot_scale, const double* x,
                        GKVecs<double> vec, GKState* st, GKWork& wk, hipStream_t s) {
  launch_resid(A, b, b_bot, bot_scale, x, vec.u_top, vec.u_bot, st, wk, s);
  launch_bwd<double, true>(A, vec.u_top, vec.u_bot, vec.v, vec.g, st, wk, true, s);
  hipLaunchKernelGGL(k_consume, dim3(1), dim3(kBlock), 0, s, st, wk.alpha_part, (int)wk.alpha_count, 0);
}

// ||A^T b||^2 -> st[0].h2 (state: beta = 1, delta = 0, init = 1).
void op_atb_norm2(const OpDesc& A, const double* b, double* tmp_n, GKState* st, GKWork& wk, hipStream_t s) {
  launch_bwd<double, false>(A, b, nullptr, nullptr, tmp_n, st, wk, false, s);
  hipLaunchKernelGGL(k_consume, dim3(1), dim3(kBlock), 0, s, st, wk.alpha_part, (int)wk.alpha_count, 0);
}

// ||b||^2 -> st[0].beta1 (state: delta = 0).
void op_norm(const OpDesc& A, const double* b, double* tmp_m, GKState* st, GKWork& wk, hipStream_t s) {
  launch_resid(A, b, nullptr, 0.0, nullptr, tmp_m, nullptr, st, wk, s);
  hipLaunchKernelGGL(k_consume, dim3(1), dim3(kBlock), 0, s, st, wk.beta_part, (int)wk.beta_count, 1);
}

// y = A x (trans = 0; y = A x - y_prev, the LSQR forward kernel with alpha =
// beta = 1, delta = 0) or y = A^T x (trans = 1), state slots as given.
void op_matvec(const OpDesc& A, int trans, const double* x, double* y, GKState* st, GKWork& wk, hipStream_t s) {
  if (!trans) {
    GKVecs<double> vec{y, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    launch_fwd<double, kFwdMatvec>(A, x, vec, st, wk, s);
  } else {
    launch_bwd<double, false>(A, x, nullptr, nullptr, y, st, wk, false, s);
  }
}

}  // namespace aplicur
