// Golub-Kahan bidiagonalisation with the LSQR Givens recurrences (Sec. 2.2)
// on the augmented, right-preconditioned operator  A~ = A_mu P^{-1},
// A_mu = [A; delta I]  (delta = sqrt(mu)), one iteration being
//
//     beta u  = A~ v   - alpha u      (forward kernel; P^{-1} v first if P != I)
//     alpha v = A~^T u - beta  v      (backward kernel; then P^{-T})
//     Givens rotation, y += (phi/rho) w, w = v - (theta/rho) w.
//
// Reductions without fences or atomics: a kernel that produces a norm writes
// one partial sum per workgroup (grids sized for full occupancy), and a
// one-workgroup "finish" kernel sums them in a fixed order and updates the
// FP64 scalar state (beta; or alpha with the Givens rotation and the
// stopping tests of Sec. 5.3.2).  Only finish kernels write the state, so the
// products read it without races.  Normalisation by 1/beta and 1/alpha is
// folded into the next consumer, and the y/w update of iteration j is applied
// by the first kernel of iteration j + 1 (or by the phase-end kernel).
#include "kernels.h"

namespace aplicur {

constexpr int kMaxGrid = 16384;

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

__device__ __forceinline__ bool stopped(const GKState* st) { return st->stop != 0; }

// ---------------------------------------------------------------- finish kernels
// One workgroup (1024 threads): sums the partials of the producing kernel in
// a fixed order and updates the state.
enum FinMode { kFinBeta = 0, kFinAlpha = 1 };

__global__ void __launch_bounds__(1024) k_finish(GKState* st, const double* part, int count, int mode) {
  __shared__ double red[1024 / kWave];
  double v = 0.0;
  for (int i = threadIdx.x; i < count; i += 1024) v += part[i];
  v = wave_sum(v);
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  if (threadIdx.x != 0) return;
  double tot = 0.0;
  for (int i = 0; i < 1024 / kWave; ++i) tot += red[i];
  GKState s = *st;
  if (s.stop) return;
  if (mode == kFinBeta) {
    const double b = sqrt(tot);
    s.pending = 0;  // the forward kernel has applied the y/w update
    s.beta = b;
    if (!(b == b) || isinf(b)) {
      s.stop = 1;
      s.reason = 6;
    } else if (b == 0.0) {
      if (s.init) {  // zero residual at the phase start: nothing to do
        s.beta1 = 0.0;
        s.stop = 1;
        s.reason = kStopExact;
      } else {
        scalar_step(s, 0.0);  // exact solution: last y update, then stop
      }
    }
  } else {
    scalar_step(s, sqrt(tot));
  }
  *st = s;
}

// ---------------------------------------------------------------- CSR products
// CSR row dot with G lanes (used by the residual kernel).
template <class TA, class V, class X>
__device__ __forceinline__ V csr_dot(const int* __restrict__ rp, const int* __restrict__ ci,
                                     const TA* __restrict__ val, const X* __restrict__ x, long long row, int lane,
                                     int G) {
  V acc = 0;
  const int b = rp[row], e = rp[row + 1];
  for (int k = b + lane; k < e; k += G) acc += (V)val[k] * (V)x[ci[k]];
  for (int off = G >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
  return acc;
}

// CSR-stream product (after Greathouse & Daga, SC'14): workgroup j owns the
// rows whose first non-zero lies in [j T, (j + 1) T) (precomputed row
// blocks rb).  The workgroup loads the products val * x[col] of all its
// non-zeros with coalesced loads into LDS, then groups of G lanes (G chosen
// from the rows per workgroup) sum each row from LDS in a fixed order and
// call epi(row, dot) once per row (lane 0 of the group).  Rows whose
// non-zeros do not fit the LDS buffer are summed straight from memory by
// the whole workgroup.  Returns nothing; the epilogue accumulates its own
// norm partial.
constexpr int kStreamT = 1024;   // target non-zeros per workgroup
constexpr int kStreamCap = 4096; // LDS products per workgroup (32 KiB)

template <class V, class TA, class X, class Epi>
__device__ __forceinline__ void csr_stream(const int* __restrict__ rb, const int* __restrict__ rp,
                                           const int* __restrict__ ci, const TA* __restrict__ val,
                                           const X* __restrict__ x, int blk, Epi&& epi) {
  __shared__ V prod[kStreamCap];
  const int r0 = rb[blk], r1 = rb[blk + 1];
  if (r0 >= r1) return;
  const int k0 = rp[r0], k1 = rp[r1];
  const int cnt = k1 - k0;
  const int rows = r1 - r0;
  if (cnt <= kStreamCap) {
#pragma unroll 4
    for (int e = threadIdx.x; e < cnt; e += kBlock) prod[e] = (V)val[k0 + e] * (V)x[ci[k0 + e]];
    __syncthreads();
    int G = 1;
    while (G < 64 && G * 2 * rows <= kBlock) G *= 2;
    const int lane = threadIdx.x % G, grp = threadIdx.x / G, ngrp = kBlock / G;
    for (int ri = grp; ri < rows; ri += ngrp) {
      const int r = r0 + ri;
      const int a = rp[r] - k0, z = rp[r + 1] - k0;
      V acc = 0;
      for (int e = a + lane; e < z; e += G) acc += prod[e];
      for (int off = G >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
      if (lane == 0) epi(r, acc);
    }
  } else {
    for (int r = r0; r < r1; ++r) {
      V acc = 0;
      for (int k = rp[r] + threadIdx.x; k < rp[r + 1]; k += kBlock) acc += (V)val[k] * (V)x[ci[k]];
      __shared__ double red[kBlock / kWave];
      double v = wave_sum((double)acc);
      __syncthreads();
      if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = v;
      __syncthreads();
      if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < kBlock / kWave; ++i) t += red[i];
        epi(r, (V)t);
      }
    }
  }
}

// Row blocks of the stream product: rb[j] = first row r with rp[r] >= j T
// (j = 0 .. nb - 1) and rb[nb] = m, nb = nnz / T + 1.
__global__ void k_row_blocks(const int* rp, long long m, int T, int* rb, int nb) {
  const long long r = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (r > m) return;
  const long long hi = (long long)rp[r] / T;
  const long long lo = (r == 0) ? 0 : (long long)rp[r - 1] / T + 1;
  for (long long j = lo; j <= hi && j < nb; ++j) rb[j] = (int)r;
  if (r == m) rb[nb] = (int)m;
}

int stream_blocks(long long nnz) { return (int)(nnz / kStreamT) + 1; }

void build_row_blocks(const int* rp, long long m, long long nnz, int* rb, hipStream_t s) {
  const int nb = stream_blocks(nnz);
  hipLaunchKernelGGL(k_row_blocks, dim3(ceil_div(m + 1, kBlock)), dim3(kBlock), 0, s, rp, m, kStreamT, rb, nb);
}

// Bottom (n-length) part of the forward kernel: u_bot update and the y/w
// update of the previous iteration.
template <class V>
__device__ __forceinline__ double fwd_bottom(long long j, const V* tin, V* u_bot, const V* v, V* w, V* y,
                                             double delta, V ts, V cu, bool pend, V cy, V cw) {
  double sq = 0.0;
  if (delta > 0.0) {
    const V ub = (V)delta * (tin[j] * ts) - cu * u_bot[j];
    u_bot[j] = ub;
    sq = (double)ub * (double)ub;
  }
  if (pend) {
    const V vj = v[j] * ts;
    const V wj = w[j];
    y[j] += cy * wj;
    w[j] = vj - cw * wj;
  }
  return sq;
}

// u_top <- A (tin / alpha) - (alpha / beta) u_top ; u_bot <- delta tin/alpha - (alpha/beta) u_bot;
// partials of ||u||^2.  `pend_ok`: apply the pending y/w update (no preconditioner).
template <class TA, class V>
__global__ void __launch_bounds__(kBlock)
    k_fwd_csr(const int* __restrict__ rb, const int* __restrict__ rp, const int* __restrict__ ci,
              const TA* __restrict__ val, long long m, long long n, const V* tin, V* u_top, V* u_bot, const V* v, V* w,
              V* y, const GKState* st, double* beta_part, int row_blocks, int pend_ok) {
  if (stopped(st)) return;
  const double alpha = st->alpha, beta = st->beta, delta = st->delta;
  const V ts = (V)(1.0 / alpha), cu = (V)(alpha / beta);
  double sq = 0.0;
  if ((int)blockIdx.x < row_blocks) {
    csr_stream<V>(rb, rp, ci, val, tin, blockIdx.x, [&](int r, V dot) {
      const V un = dot * ts - cu * u_top[r];
      u_top[r] = un;
      sq += (double)un * (double)un;
    });
  } else {
    const bool pend = pend_ok && st->pending;
    const V cy = (V)st->coef_y, cw = (V)st->coef_w;
    const int nb = gridDim.x - row_blocks;
    for (long long j = (long long)(blockIdx.x - row_blocks) * kBlock + threadIdx.x; j < n; j += (long long)nb * kBlock)
      sq += fwd_bottom<V>(j, tin, u_bot, v, w, y, delta, ts, cu, pend, cy, cw);
  }
  const double bs = block_sum(sq);
  if (threadIdx.x == 0) beta_part[blockIdx.x] = bs;
}

// Dense row-major A: one wave per row.
template <class TA, class V>
__global__ void __launch_bounds__(kBlock)
    k_fwd_dense(const TA* __restrict__ A, long long m, long long n, long long ld, const V* tin, V* u_top, V* u_bot,
                const V* v, V* w, V* y, const GKState* st, double* beta_part, int row_blocks, int pend_ok) {
  if (stopped(st)) return;
  const double alpha = st->alpha, beta = st->beta, delta = st->delta;
  const V ts = (V)(1.0 / alpha), cu = (V)(alpha / beta);
  double sq = 0.0;
  if ((int)blockIdx.x < row_blocks) {
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
    const bool pend = pend_ok && st->pending;
    const V cy = (V)st->coef_y, cw = (V)st->coef_w;
    const int nb = gridDim.x - row_blocks;
    for (long long j = (long long)(blockIdx.x - row_blocks) * kBlock + threadIdx.x; j < n; j += (long long)nb * kBlock)
      sq += fwd_bottom<V>(j, tin, u_bot, v, w, y, delta, ts, cu, pend, cy, cw);
  }
  const double bs = block_sum(sq);
  if (threadIdx.x == 0) beta_part[blockIdx.x] = bs;
}

// Backward epilogue: g = (dot + delta u_bot) / beta.  PLAIN: v_raw <- g -
// (beta/alpha) v_raw (g at the phase start); otherwise g is stored for P^{-T}.
// Returns the squared entry for the norm partials.
template <class V, bool PLAIN>
__device__ __forceinline__ double bwd_epilogue(long long j, V dot, const V* u_bot, V* v, V* g, double delta, V ib,
                                               V cv, int init) {
  V gj = dot * ib;
  if (delta > 0.0) gj += (V)delta * u_bot[j] * ib;
  if (PLAIN) {
    const V vn = init ? gj : gj - cv * v[j];
    v[j] = vn;
    return (double)vn * (double)vn;
  } else {
    g[j] = gj;
    return (double)gj * (double)gj;
  }
}

template <class TA, class V, bool PLAIN>
__global__ void __launch_bounds__(kBlock)
    k_bwd_csr(const int* __restrict__ trb, const int* __restrict__ tp, const int* __restrict__ ti,
              const TA* __restrict__ tv, long long n, const V* u_top, const V* u_bot, V* v, V* g, const GKState* st,
              double* alpha_part) {
  if (stopped(st)) return;
  const double beta = st->beta, alpha = st->alpha, delta = st->delta;
  const int init = st->init;
  const V ib = (V)(1.0 / beta), cv = (V)(beta / alpha);
  double sq = 0.0;
  csr_stream<V>(trb, tp, ti, tv, u_top, blockIdx.x,
                [&](int j, V dot) { sq += bwd_epilogue<V, PLAIN>(j, dot, u_bot, v, g, delta, ib, cv, init); });
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
                    const GKState* st, double* alpha_part) {
  if (stopped(st)) return;
  const double beta = st->beta, alpha = st->alpha, delta = st->delta;
  const int init = st->init;
  const V ib = (V)(1.0 / beta), cv = (V)(beta / alpha);
  double sq = 0.0;
  for (long long j = (long long)blockIdx.x * kBlock + threadIdx.x; j < n; j += (long long)gridDim.x * kBlock) {
    double acc = 0.0;
    for (int c = 0; c < chunks; ++c) acc += part[(long long)c * n + j];
    sq += bwd_epilogue<V, PLAIN>(j, (V)acc, u_bot, v, g, delta, ib, cv, init);
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

// t = v_raw + V c  (= P^{-1} v_raw) and the pending y/w update.
template <class V>
__global__ void __launch_bounds__(kBlock)
    k_pa_fwd(const double* __restrict__ Vh, long long n, int ell, long long ldv, const double* __restrict__ c,
             const V* v, V* t, V* w, V* y, const GKState* st) {
  if (stopped(st)) return;
  const bool pend = st->pending;
  const double cy = st->coef_y, cw = st->coef_w, ia = 1.0 / st->alpha;
  const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  constexpr int rpb = kBlock / kWave;
  for (long long i = (long long)blockIdx.x * rpb + wv; i < n; i += (long long)gridDim.x * rpb) {
    const double dot = vrow_dot(Vh, ldv, ell, c, i, lane);
    if (lane == 0) {
      const V vi = v[i];
      t[i] = (V)((double)vi + dot);
      if (pend) {
        const V wi = w[i];
        y[i] += (V)cy * wi;
        w[i] = (V)((double)vi * ia) - (V)cw * wi;
      }
    }
  }
}

// v_raw <- (g + V c) - (beta/alpha) v_raw  (g + V c at the phase start);
// partials of ||v_raw||^2.
template <class V>
__global__ void __launch_bounds__(kBlock)
    k_pa_bwd(const double* __restrict__ Vh, long long n, int ell, long long ldv, const double* __restrict__ c,
             const V* g, V* v, const GKState* st, double* alpha_part) {
  if (stopped(st)) return;
  const int init = st->init;
  const double cv = st->beta / st->alpha;
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

// ---------------------------------------------------------------- phase start / end
// r_top = b - A x (FP64, values widened), r_bot = bot_scale b_bot - delta x;
// partials of ||r||^2.
template <class TA>
__global__ void __launch_bounds__(kBlock)
    k_resid_csr(const int* __restrict__ rp, const int* __restrict__ ci, const TA* __restrict__ val, long long m,
                long long n, const double* __restrict__ b, const double* b_bot, double bot_scale, const double* x,
                int x_zero, double* r_top, double* r_bot, const GKState* st, double* beta_part, int G,
                int row_blocks) {
  const double delta = st->delta;
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
  const double delta = st->delta;
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

// Phase end: the last pending y update (w is not needed afterwards).
template <class V>
__global__ void k_finalize(long long n, V* y, const V* w, const GKState* st) {
  if (!st->pending) return;
  const V cy = (V)st->coef_y;
  for (long long j = (long long)blockIdx.x * kBlock + threadIdx.x; j < n; j += (long long)gridDim.x * kBlock)
    y[j] += cy * w[j];
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
  if (A.csr) return (unsigned)stream_blocks(A.nnz);
  return clamp_grid((A.m + 3) / 4);
}
static unsigned bwd_grid(const OpDesc& A) {
  if (A.csr) return (unsigned)stream_blocks(A.nnz);
  return clamp_grid(ceil_div(A.n, kBlock));
}
static unsigned rows_grid(long long n) { return clamp_grid((n + 3) / 4); }

static void finish(GKState* st, GKWork& wk, int mode, hipStream_t s) {
  if (mode == kFinBeta)
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, st, wk.beta_part, (int)wk.beta_count, mode);
  else
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, st, wk.alpha_part, (int)wk.alpha_count, mode);
}

template <class V>
static void launch_fwd(const OpDesc& A, const V* tin, GKVecs<V> vec, const GKState* st, GKWork& wk, int pend_ok,
                       hipStream_t s) {
  const unsigned rb = fwd_row_blocks(A);
  const unsigned grid = rb + nbottom(A.n);
  if (A.csr) {
    if (A.f64)
      hipLaunchKernelGGL((k_fwd_csr<double, V>), dim3(grid), dim3(kBlock), 0, s, A.rb, A.row_ptr, A.col_idx,
                         (const double*)A.val, A.m, A.n, tin, vec.u_top, vec.u_bot, vec.v, vec.w, vec.y, st,
                         wk.beta_part, (int)rb, pend_ok);
    else
      hipLaunchKernelGGL((k_fwd_csr<float, V>), dim3(grid), dim3(kBlock), 0, s, A.rb, A.row_ptr, A.col_idx,
                         (const float*)A.val, A.m, A.n, tin, vec.u_top, vec.u_bot, vec.v, vec.w, vec.y, st,
                         wk.beta_part, (int)rb, pend_ok);
  } else {
    if (A.f64)
      hipLaunchKernelGGL((k_fwd_dense<double, V>), dim3(grid), dim3(kBlock), 0, s, (const double*)A.val, A.m, A.n,
                         A.ld, tin, vec.u_top, vec.u_bot, vec.v, vec.w, vec.y, st, wk.beta_part, (int)rb, pend_ok);
    else
      hipLaunchKernelGGL((k_fwd_dense<float, V>), dim3(grid), dim3(kBlock), 0, s, (const float*)A.val, A.m, A.n,
                         A.ld, tin, vec.u_top, vec.u_bot, vec.v, vec.w, vec.y, st, wk.beta_part, (int)rb, pend_ok);
  }
  wk.beta_count = grid;
}

template <class V, bool PLAIN>
static void launch_bwd(const OpDesc& A, const V* u_top, const V* u_bot, V* v, V* g, const GKState* st, GKWork& wk,
                       hipStream_t s) {
  if (A.csr) {
    const unsigned grid = bwd_grid(A);
    if (A.f64)
      hipLaunchKernelGGL((k_bwd_csr<double, V, PLAIN>), dim3(grid), dim3(kBlock), 0, s, A.t_rb, A.t_ptr, A.t_idx,
                         (const double*)A.t_val, A.n, u_top, u_bot, v, g, st, wk.alpha_part);
    else
      hipLaunchKernelGGL((k_bwd_csr<float, V, PLAIN>), dim3(grid), dim3(kBlock), 0, s, A.t_rb, A.t_ptr, A.t_idx,
                         (const float*)A.t_val, A.n, u_top, u_bot, v, g, st, wk.alpha_part);
    wk.alpha_count = grid;
  } else {
    const long long rpc = (A.m + A.chunks - 1) / A.chunks;
    dim3 g1(ceil_div(A.n, kBlock), A.chunks);
    if (A.f64)
      hipLaunchKernelGGL((k_bwd_dense_part<double, V>), g1, dim3(kBlock), 0, s, (const double*)A.val, A.m, A.n, A.ld,
                         u_top, A.part, rpc, st);
    else
      hipLaunchKernelGGL((k_bwd_dense_part<float, V>), g1, dim3(kBlock), 0, s, (const float*)A.val, A.m, A.n, A.ld,
                         u_top, A.part, rpc, st);
    const unsigned grid = bwd_grid(A);
    hipLaunchKernelGGL((k_bwd_dense_red<V, PLAIN>), dim3(grid), dim3(kBlock), 0, s, A.part, A.chunks, A.n, u_bot, v,
                       g, st, wk.alpha_part);
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
static void launch_pa_bwd(const PrecDesc& P, long long n, const V* g, V* v, const GKState* st, GKWork& wk,
                          hipStream_t s) {
  const unsigned rg = rows_grid(n);
  hipLaunchKernelGGL((k_pa_bwd<V>), dim3(rg), dim3(kBlock), 0, s, P.V, n, P.ell, P.ldv, P.c, g, v, st,
                     wk.alpha_part);
  wk.alpha_count = rg;
}

template <class V>
void gk_iteration(const OpDesc& A, const PrecDesc* P, GKVecs<V> vec, GKState* st, GKWork& wk, hipStream_t s) {
  if (!P) {
    launch_fwd<V>(A, vec.v, vec, st, wk, 1, s);
    finish(st, wk, kFinBeta, s);
    launch_bwd<V, true>(A, vec.u_top, vec.u_bot, vec.v, vec.g, st, wk, s);
    finish(st, wk, kFinAlpha, s);
    return;
  }
  launch_pa_c<V>(*P, A.n, vec.v, st, s);
  hipLaunchKernelGGL((k_pa_fwd<V>), dim3(rows_grid(A.n)), dim3(kBlock), 0, s, P->V, A.n, P->ell, P->ldv, P->c, vec.v,
                     vec.t, vec.w, vec.y, (const GKState*)st);
  launch_fwd<V>(A, vec.t, vec, st, wk, 0, s);
  finish(st, wk, kFinBeta, s);
  launch_bwd<V, false>(A, vec.u_top, vec.u_bot, vec.v, vec.g, st, wk, s);
  launch_pa_c<V>(*P, A.n, vec.g, st, s);
  launch_pa_bwd<V>(*P, A.n, vec.g, vec.v, st, wk, s);
  finish(st, wk, kFinAlpha, s);
}

static void launch_resid(const OpDesc& A, const double* b, const double* b_bot, double bot_scale, const double* x,
                         double* r_top, double* r_bot, const GKState* st, GKWork& wk, hipStream_t s) {
  const int x_zero = (x == nullptr);
  const unsigned rb = A.csr ? clamp_grid((A.m + (kBlock / A.group) - 1) / (kBlock / A.group)) : fwd_row_blocks(A);
  const unsigned grid = rb + nbottom(A.n);
  if (A.csr) {
    if (A.f64)
      hipLaunchKernelGGL((k_resid_csr<double>), dim3(grid), dim3(kBlock), 0, s, A.row_ptr, A.col_idx,
                         (const double*)A.val, A.m, A.n, b, b_bot, bot_scale, x, x_zero, r_top, r_bot, st,
                         wk.beta_part, A.group, (int)rb);
    else
      hipLaunchKernelGGL((k_resid_csr<float>), dim3(grid), dim3(kBlock), 0, s, A.row_ptr, A.col_idx,
                         (const float*)A.val, A.m, A.n, b, b_bot, bot_scale, x, x_zero, r_top, r_bot, st,
                         wk.beta_part, A.group, (int)rb);
  } else {
    if (A.f64)
      hipLaunchKernelGGL((k_resid_dense<double>), dim3(grid), dim3(kBlock), 0, s, (const double*)A.val, A.m, A.n,
                         A.ld, b, b_bot, bot_scale, x, x_zero, r_top, r_bot, st, wk.beta_part, (int)rb);
    else
      hipLaunchKernelGGL((k_resid_dense<float>), dim3(grid), dim3(kBlock), 0, s, (const float*)A.val, A.m, A.n,
                         A.ld, b, b_bot, bot_scale, x, x_zero, r_top, r_bot, st, wk.beta_part, (int)rb);
  }
  wk.beta_count = grid;
}

template <class V>
void gk_phase_init(const OpDesc& A, const PrecDesc* P, const double* b, const double* b_bot, double bot_scale,
                   const double* x, GKVecs<V> vec, double* r_top64, double* r_bot64, GKState* st, GKWork& wk,
                   hipStream_t s) {
  static_assert(sizeof(V) == 8, "only the FP64 vector path is implemented here");
  launch_resid(A, b, b_bot, bot_scale, x, r_top64, r_bot64, st, wk, s);
  finish(st, wk, kFinBeta, s);
  fill_zero<V>(vec.y, A.n, s);
  fill_zero<V>(vec.w, A.n, s);
  if (!P) {
    launch_bwd<V, true>(A, (const V*)r_top64, (const V*)r_bot64, vec.v, vec.g, st, wk, s);
  } else {
    launch_bwd<V, false>(A, (const V*)r_top64, (const V*)r_bot64, vec.v, vec.g, st, wk, s);
    launch_pa_c<V>(*P, A.n, vec.g, st, s);
    launch_pa_bwd<V>(*P, A.n, vec.g, vec.v, st, wk, s);
  }
  finish(st, wk, kFinAlpha, s);
}

template <class V>
void gk_phase_finish(const OpDesc& A, const PrecDesc* P, GKVecs<V> vec, double* x, GKState* st, hipStream_t s) {
  const unsigned g = clamp_grid(ceil_div(A.n, kBlock));
  hipLaunchKernelGGL((k_finalize<V>), dim3(g), dim3(kBlock), 0, s, A.n, vec.y, vec.w, (const GKState*)st);
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

// ||A_mu^T r||^2 -> st->h2 for r = [b - A x; bot_scale b_bot - delta x]: the
// plain phase start (its initial scalar step stores (alpha_1 beta_1)^2).
void gk_normal_residual(const OpDesc& A, const double* b, const double* b_bot, double bot_scale, const double* x,
                        GKVecs<double> vec, GKState* st, GKWork& wk, hipStream_t s) {
  launch_resid(A, b, b_bot, bot_scale, x, vec.u_top, vec.u_bot, st, wk, s);
  finish(st, wk, kFinBeta, s);
  launch_bwd<double, true>(A, vec.u_top, vec.u_bot, vec.v, vec.g, st, wk, s);
  finish(st, wk, kFinAlpha, s);
}

// ||A^T b||^2 -> st->h2 (state: beta = 1, delta = 0, init = 1).
void op_atb_norm2(const OpDesc& A, const double* b, double* tmp_n, GKState* st, GKWork& wk, hipStream_t s) {
  launch_bwd<double, false>(A, b, nullptr, nullptr, tmp_n, st, wk, s);
  finish(st, wk, kFinAlpha, s);
}

// ||b|| -> st->beta (state: delta = 0, init = 1).
void op_norm(const OpDesc& A, const double* b, double* tmp_m, GKState* st, GKWork& wk, hipStream_t s) {
  launch_resid(A, b, nullptr, 0.0, nullptr, tmp_m, nullptr, st, wk, s);
  finish(st, wk, kFinBeta, s);
}

// y = A x - y_prev (trans = 0; the LSQR forward kernel with alpha = beta = 1,
// delta = 0) or y = A^T x (trans = 1); state as given, not modified.
void op_matvec(const OpDesc& A, int trans, const double* x, double* y, GKState* st, GKWork& wk, hipStream_t s) {
  if (!trans) {
    GKVecs<double> vec{y, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    launch_fwd<double>(A, x, vec, st, wk, 0, s);
  } else {
    launch_bwd<double, false>(A, x, nullptr, nullptr, y, st, wk, s);
  }
}

}  // namespace aplicur
