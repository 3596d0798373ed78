// Golub-Kahan bidiagonalisation with the LSQR Givens recurrences (Sec. 2.2)
// on the augmented, right-preconditioned operator  A~ = A_mu P^{-1},
// A_mu = [A; delta I]  (delta = sqrt(mu)), one iteration being
//
//     beta u  = A~ v   - alpha u      (forward kernel; P^{-1} v first if P != I)
//     alpha v = A~^T u - beta  v      (backward kernel; then P^{-T} = P^{-1})
//     Givens rotation, y += (phi/rho) w, w = v - (theta/rho) w.
//
// Reductions without fences, atomics or extra launches.  A kernel that
// produces a norm writes one partial sum per workgroup.  Every workgroup of
// the kernel that consumes the norm loads those partials together with its
// own first operands, sums them in a fixed order (thread-strided sums, a
// shuffle tree, the waves in order) so that all workgroups hold the
// bitwise-identical scalar, and advances its private copy of the FP64 state
// with it (the same arithmetic in every thread).  The state has two slots:
// slot 0 is written by the kernel that finishes alpha and takes the Givens
// step with the stopping tests of Sec. 5.3.2, slot 1 by the kernel that
// finishes beta; a kernel reads only the slot it does not write, and only
// workgroup 0 stores, so there is no race.  A stopped state is copied
// forward by the next kernels until the host sees it.  Normalisation by
// 1/beta and 1/alpha is folded into the consumers, and the y/w update of
// iteration j is applied by the first kernel of iteration j + 1, which on
// stopping applies the last y update itself.
#include <hip/hip_ext.h>

#include <algorithm>
#include <vector>

#include "gk_scalar.h"
#include "kernels.h"

namespace aplicur {

constexpr int kMaxGrid = 4096;                // grid-stride kernels
constexpr int kStreamCap = 2048;              // CSR-stream: LDS products per workgroup
constexpr int kPer = kStreamCap / kBlock;     // products per thread
constexpr int kRowsMaxGrid = 512;             // row-wise P-apply kernels (their partials are re-read)

// ---------------------------------------------------------------- consumer reductions
// This thread's share of the producer partials part[0..count), in a fixed
// order.  load() issues the first kShare * kBlock loads without using their
// values (indices clamped into range), so that the caller's next loads issue
// before the first wait; sum() masks and adds them.  Partials beyond the first
// round (grids above kShare * kBlock workgroups) are summed at once.
constexpr int kShare = 8;
template <int NT = kBlock, int KS = kShare>
struct ShareT {
  double t[KS];
  double rest;
  int count;
  __device__ __forceinline__ void load(const double* __restrict__ part, int count_) {
    count = part ? count_ : 0;
    rest = 0.0;
    if (count <= 0) return;
#pragma unroll
    for (int q = 0; q < KS; ++q) t[q] = part[min(q * NT + (int)threadIdx.x, count - 1)];
    for (int i = KS * NT + threadIdx.x; i < count; i += NT) rest += part[i];
  }
  __device__ __forceinline__ double sum() const {
    double v = 0.0;
    if (count <= 0) return v;
#pragma unroll
    for (int q = 0; q < KS; ++q) v += (q * NT + (int)threadIdx.x < count) ? t[q] : 0.0;
    return v + rest;
  }
};
using Share = ShareT<>;

// Wave sums into red[]; the caller's barrier follows.
template <class SH>
__device__ __forceinline__ void publish(const SH& sh, double* red) {
  const double v = wave_sum(sh.sum());
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = v;
}

template <int NT = kBlock>
__device__ __forceinline__ double settled(const double* red) {
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < NT / kWave; ++i) t += red[i];
  return t;
}

// Sum over a workgroup of NT threads; valid in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum_t(double v) {
  __shared__ double red[NT / kWave];
  v = wave_sum(v);
  __syncthreads();
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  return threadIdx.x == 0 ? settled<NT>(red) : 0.0;
}

__device__ __forceinline__ void store_state(GKState* out, const GKState& s) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *out = s;
}

// ---------------------------------------------------------------- CSR-stream product
// After Greathouse & Daga (SC'14): workgroup j owns the rows whose first
// non-zero lies in [j T, (j + 1) T) (row blocks rbk[j] = {first row, its
// first non-zero}).  In one dependent stage after rbk it loads its
// non-zeros' values and columns, and each group of G lanes loads the
// pointers and two epilogue operands (`pre`) of its first row; then it
// gathers x[col], stores the products in LDS and, after the one barrier
// (shared with the producer-partial reduction and `settle`, which advances
// the state and may end the kernel), the groups sum their rows in a fixed
// order and call epi(row, dot, pre0, pre1) in lane 0.  Row blocks whose
// non-zeros exceed the LDS buffer (a row longer than about T) take a direct
// workgroup-per-row path.  Returns false when `settle` ended the kernel.
// The caller loads the row-block bounds a = rbk[j], b = rbk[j + 1] in its
// first stage, together with the producer partials and the state.
struct RowBlk {
  int r0, k0;
};

template <class V, class TA, class X, class SH, class Pre, class Settle, class Epi>
__device__ __forceinline__ bool csr_stream(RowBlk a, RowBlk b, const int* __restrict__ rp,
                                           const int* __restrict__ ci, const TA* __restrict__ val,
                                           const X* __restrict__ x, const SH& share, Pre&& pre,
                                           Settle&& settle, Epi&& epi) {
  __shared__ V prod[kStreamCap];
  __shared__ double red[kBlock / kWave];
  const int r0 = a.r0, k0 = a.k0, rows = b.r0 - a.r0, cnt = b.k0 - a.k0;
  const bool staged = cnt <= kStreamCap;
  int G = 1;
  while (G < 64 && G * 2 * rows <= kBlock) G *= 2;
  const int lane = threadIdx.x % G, grp = threadIdx.x / G, ngrp = kBlock / G;
  // Loads without branches (indices clamped into range, the matrix has at
  // least one row), so that they all issue before the first wait.
  const int rr = rows > 0 ? r0 + min(grp, rows - 1) : 0;
  int lo = rp[rr] - k0, hi = rp[rr + 1] - k0;
  V q0, q1;
  pre(rr, q0, q1);
  if (staged && cnt > 0) {
    int cidx[kPer];
    TA vv[kPer];
    V xv[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = threadIdx.x + q * kBlock;
      const int idx = k0 + min(e, cnt - 1);
      cidx[q] = ci[idx];
      const TA t = val[idx];
      vv[q] = e < cnt ? t : (TA)0;
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) xv[q] = (V)x[cidx[q]];
#pragma unroll
    for (int q = 0; q < kPer; ++q) prod[threadIdx.x + q * kBlock] = (V)vv[q] * xv[q];
  }
  publish(share, red);
  __syncthreads();
  if (!settle(settled(red))) return false;
  if (staged) {
    for (int ri = grp; ri < rows; ri += ngrp) {
      if (ri != grp) {
        lo = rp[r0 + ri] - k0;
        hi = rp[r0 + ri + 1] - k0;
        pre(r0 + ri, q0, q1);
      }
      V acc = 0;
      for (int e = lo + lane; e < hi; e += G) acc += prod[e];
      for (int off = G >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
      if (lane == 0) epi(r0 + ri, acc, q0, q1);
    }
  } else {
    __shared__ double red2[kBlock / kWave];
    for (int r = r0; r < r0 + rows; ++r) {
      V acc = 0;
      const int kb = rp[r], ke = rp[r + 1];
      for (int k = kb + threadIdx.x; k < ke; k += kBlock) acc += (V)val[k] * (V)x[ci[k]];
      const double v = wave_sum((double)acc);
      __syncthreads();
      if (threadIdx.x % kWave == 0) red2[threadIdx.x / kWave] = v;
      __syncthreads();
      if (threadIdx.x == 0) {
        V p0 = 0, p1 = 0;
        pre(r, p0, p1);
        epi(r, (V)settled(red2), p0, p1);
      }
    }
  }
  return true;
}

// rbk[j] = {first row r with rp[r] >= j T, rp[r]} (j < nb), rbk[nb] = {m, nnz},
// nb = nnz / T + 1 (the last workgroup also owns trailing empty rows).
__global__ void k_row_blocks(const int* rp, long long m, int T, RowBlk* rbk, int nb) {
  const long long r = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (r > m) return;
  const long long hi = (long long)rp[r] / T;
  const long long lo = (r == 0) ? 0 : (long long)rp[r - 1] / T + 1;
  for (long long j = lo; j <= hi && j < nb; ++j) rbk[j] = RowBlk{(int)r, rp[r]};
  if (r == m) rbk[nb] = RowBlk{(int)m, rp[m]};
}

// Non-zeros per workgroup T: the grid of a product (nnz / T + 1 row blocks
// plus the bottom blocks) should be resident at once (about 7 workgroups per
// CU at this kernel's LDS and register use), so T grows from 1024 with nnz up
// to 1536, which leaves LDS room for a row tail of 512 non-zeros.
int stream_t(long long nnz) {
  static const int cus = []() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
      v = 256;
    return v;
  }();
  const long long resident = 7LL * cus - 64;
  long long t = (nnz + resident - 1) / resident;
  if (t < 1024) t = 1024;
  if (t > 1536) t = 1536;
  return (int)t;
}
int stream_blocks(long long nnz, int T) { return (int)(nnz / T) + 1; }
long long row_block_words(long long nnz, int T) { return 2LL * (stream_blocks(nnz, T) + 1); }

void build_row_blocks(const int* rp, long long m, long long nnz, int T, int* rb, hipStream_t s) {
  const int nb = stream_blocks(nnz, T);
  hipLaunchKernelGGL(k_row_blocks, dim3(ceil_div(m + 1, kBlock)), dim3(kBlock), 0, s, rp, m, T, (RowBlk*)rb, nb);
}

// ---------------------------------------------------------------- forward kernels
template <class V>
__device__ __forceinline__ void final_y(long long n, V* y, const V* w, const GKState& s, long long first,
                                        long long stride) {
  if (!s.pending) return;
  const V cy = (V)s.coef_y;
  for (long long j = first; j < n; j += stride) y[j] += cy * w[j];
}

// Bottom rows of the forward kernel: u_bot <- delta tin/alpha - (alpha/beta) u_bot,
// and the y/w update of the previous iteration (PLAIN).
template <class V, int MODE>
__device__ __forceinline__ double fwd_bottom(long long n, const V* tin, V* u_bot, const V* v, V* w, V* y,
                                             GKState& s, GKState* __restrict__ st_out, const Share& share,
                                             long long first,
                                             long long stride) {
  __shared__ double red[kBlock / kWave];
  const double delta = s.delta;
  V t0 = 0, ub0 = 0, v0 = 0, w0 = 0, y0 = 0;
  const long long j0 = first < n ? first : n - 1;  // in range (n >= 1); unused if first >= n
  if (MODE != kFwdMatvec) {
    t0 = tin[j0];
    ub0 = u_bot[j0];
  }
  if (MODE == kFwdPlain) {
    v0 = v[j0];
    w0 = w[j0];
    y0 = y[j0];
  }
  publish(share, red);
  __syncthreads();
  if (MODE == kFwdPlain) {
    scalar_step(s, sqrt(settled(red)));
    store_state(st_out, s);
    if (s.stop) {
      final_y<V>(n, y, w, s, first, stride);
      return -1.0;
    }
  }
  const V ts = (V)(1.0 / s.alpha), cu = (V)(s.alpha / s.beta);
  const bool pend = (MODE == kFwdPlain) && s.pending;
  const V cy = (V)s.coef_y, cw = (V)s.coef_w;
  double sq = 0.0;
  for (long long j = first; j < n; j += stride) {
    V tj = t0, ubj = ub0, vj = v0, wj = w0, yj = y0;
    if (j != first) {
      if (delta > 0.0) {
        tj = tin[j];
        ubj = u_bot[j];
      }
      if (pend) {
        vj = v[j];
        wj = w[j];
        yj = y[j];
      }
    }
    if (delta > 0.0) {
      const V ub = (V)delta * (tj * ts) - cu * ubj;
      u_bot[j] = ub;
      sq += (double)ub * (double)ub;
    }
    if (pend) {
      y[j] = yj + cy * wj;
      w[j] = vj * ts - cw * wj;
    }
  }
  return sq;
}

// u_top <- A (tin / alpha) - (alpha / beta) u_top ; u_bot likewise; partials of ||u||^2.
template <class TA, class V, int MODE>
__global__ void __launch_bounds__(kBlock)
    k_fwd_csr(const RowBlk* __restrict__ rbk, const int* __restrict__ rp, const int* __restrict__ ci,
              const TA* __restrict__ val, long long n, const V* tin, V* u_top, V* u_bot, const V* v, V* w, V* y,
              const GKState* __restrict__ st_in, GKState* __restrict__ st_out, const double* alpha_part,
              int alpha_count, double* beta_part, int row_blocks) {
  const bool rows_part = (int)blockIdx.x < row_blocks;
  RowBlk ra{0, 0}, rb{0, 0};
  if (rows_part) {
    ra = rbk[blockIdx.x];
    rb = rbk[blockIdx.x + 1];
  }
  GKState s = *st_in;
  Share share;
  share.load(MODE == kFwdPlain ? alpha_part : nullptr, alpha_count);
  if (MODE != kFwdMatvec && s.stop) {
    if (MODE == kFwdPlain) store_state(st_out, s);
    return;
  }
  double sq = 0.0;
  if (rows_part) {
    V ts = 0, cu = 0;
    const bool ran = csr_stream<V>(
        ra, rb, rp, ci, val, tin, share,
        [&](int r, V& q0, V& q1) {
          q0 = u_top[r];
          q1 = 0;
        },
        [&](double total) {
          if (MODE == kFwdPlain) {
            scalar_step(s, sqrt(total));
            store_state(st_out, s);
          }
          ts = (V)(1.0 / s.alpha);
          cu = (V)(s.alpha / s.beta);
          return !s.stop;
        },
        [&](int r, V dot, V q0, V) {
          const V un = dot * ts - cu * q0;
          u_top[r] = un;
          sq += (double)un * (double)un;
        });
    if (!ran) return;
  } else {
    const long long stride = (long long)(gridDim.x - row_blocks) * kBlock;
    sq = fwd_bottom<V, MODE>(n, tin, u_bot, v, w, y, s, st_out, share,
                             (long long)(blockIdx.x - row_blocks) * kBlock + threadIdx.x, stride);
    if (MODE == kFwdPlain && s.stop) return;
  }
  const double bs = block_sum(sq);
  if (threadIdx.x == 0) beta_part[blockIdx.x] = bs;
}

// A x with x resident in LDS (n values fit one workgroup's LDS): one
// 1024-thread workgroup per CU and row block (rows starting in its window of
// nnz / grid non-zeros).  Stage 1 loads x into LDS together with the row-block
// pair, the producer partials and the state; each thread then takes one row
// (rows beyond 1024 loop), loads its pointers and its first kLxChunk values
// and columns at once, and sums val * x[col] from LDS in row order.  The
// workgroup also owns a slice of the n bottom rows (u_bot and the y/w update).
constexpr int kLxT = 1024;
constexpr int kLxChunk = 12;

template <class V>
struct Wide16;
template <>
struct Wide16<double> {
  using type = double2;
};
template <>
struct Wide16<float> {
  using type = float4;
};

// x (n entries, n sizeof(V) <= kLxMaxBytes) -> xs in LDS in one batch of loads
// per thread: 16-byte loads when x is 16-byte aligned (ten per thread cover
// the largest n; they move the copy at about 1.5 times the rate of 8-byte
// loads), else batches of single-entry loads.  Loads issued before the call
// stay in flight.
template <class V>
__device__ __forceinline__ void x_to_lds(const V* __restrict__ x, long long n, V* xs) {
  using V16 = typename Wide16<V>::type;
  constexpr int kW = (int)(16 / sizeof(V));
  const long long np = n / kW;
  if ((((unsigned long long)x) & 15ull) == 0 && np > 0) {
    constexpr int kB = (int)((kLxMaxBytes / 16 + kLxT - 1) / kLxT);
    const V16* x16 = (const V16*)x;
    V16* xs16 = (V16*)xs;
    V16 t[kB];
#pragma unroll
    for (int q = 0; q < kB; ++q) t[q] = x16[min((long long)threadIdx.x + (long long)q * kLxT, np - 1)];
#pragma unroll
    for (int q = 0; q < kB; ++q) {
      const long long i = (long long)threadIdx.x + (long long)q * kLxT;
      if (i < np) xs16[i] = t[q];
    }
    const long long i = np * kW + threadIdx.x;  // the last n mod kW entries
    if (i < n) xs[i] = x[i];
  } else {
    // unaligned x (a view into a larger tensor): batches of 8 entries
    for (long long base = threadIdx.x; base < n; base += (long long)kLxT * 8) {
      V t[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) t[q] = x[min(base + (long long)q * kLxT, n - 1)];
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (base + (long long)q * kLxT < n) xs[base + (long long)q * kLxT] = t[q];
    }
  }
}

template <class TA, class V, int MODE>
__global__ void __launch_bounds__(kLxT)
    k_fwd_csr_lx(const RowBlk* __restrict__ rbk, const int* __restrict__ rp, const int* __restrict__ ci,
                 const TA* __restrict__ val, long long n, const V* tin, V* u_top, V* u_bot, const V* v, V* w, V* y,
                 const GKState* __restrict__ st_in, GKState* __restrict__ st_out, const double* alpha_part,
                 int alpha_count, double* beta_part) {
  extern __shared__ __align__(16) double lx_raw[];
  V* xs = (V*)lx_raw;
  __shared__ double red[kLxT / kWave];
  const RowBlk ra = rbk[blockIdx.x], rb = rbk[blockIdx.x + 1];
  GKState s = *st_in;
  const double delta = st_in->delta;
  ShareT<kLxT, 2> share;
  share.load(MODE == kFwdPlain ? alpha_part : nullptr, alpha_count);
  if (MODE != kFwdMatvec && s.stop) {
    if (MODE == kFwdPlain) store_state(st_out, s);
    return;
  }
  // bottom slice [j0, j1) of the n rows
  const long long per = (n + gridDim.x - 1) / gridDim.x;
  const long long j0 = (long long)blockIdx.x * per, j1 = min(n, j0 + per);
  const long long jb = j0 + threadIdx.x;
  V bt = 0, bub = 0, bv = 0, bw = 0, by = 0;
  if (MODE != kFwdMatvec && jb < j1) {
    bt = tin[jb];
    bub = u_bot[jb];
    if (MODE == kFwdPlain) {
      bv = v[jb];
      bw = w[jb];
      by = y[jb];
    }
  }
  x_to_lds(tin, n, xs);
  const int r0 = ra.r0, rows = rb.r0 - ra.r0;
  double sq = 0.0;
  bool go = true;
  V ts = 0, cu = 0, cy = 0, cw = 0;
  bool pend = false;
  for (int rbase = 0; rbase < rows || rbase == 0; rbase += kLxT) {
    const int ri = rbase + threadIdx.x;
    const bool mine = ri < rows;
    const int r = r0 + (mine ? ri : 0);
    int k = 0, kend = 0;
    V uo = 0;
    if (mine) {
      k = rp[r];
      kend = rp[r + 1];
      uo = u_top[r];
    }
    int cidx[kLxChunk];
    TA vv[kLxChunk];
#pragma unroll
    for (int q = 0; q < kLxChunk; ++q) {
      const int e = min(k + q, max(kend - 1, 0));
      cidx[q] = mine && k + q < kend ? ci[e] : 0;
      vv[q] = mine && k + q < kend ? val[e] : (TA)0;
    }
    if (rbase == 0) {
      // x in LDS and the producer reduction: one barrier
      publish(share, red);
      __syncthreads();
      if (MODE == kFwdPlain) {
        scalar_step(s, sqrt(settled<kLxT>(red)));
        store_state(st_out, s);
        if (s.stop) {
          if (jb < j1 && s.pending) y[jb] = by + (V)s.coef_y * bw;
          go = false;
        }
      }
      ts = (V)(1.0 / s.alpha);
      cu = (V)(s.alpha / s.beta);
      pend = (MODE == kFwdPlain) && s.pending;
      cy = (V)s.coef_y;
      cw = (V)s.coef_w;
    }
    if (!go) return;
    V acc = 0;
#pragma unroll
    for (int q = 0; q < kLxChunk; ++q) acc += (V)vv[q] * xs[cidx[q]];
    for (int e = k + kLxChunk; e < kend; ++e) acc += (V)val[e] * xs[ci[e]];
    if (mine) {
      const V un = acc * ts - cu * uo;
      u_top[r] = un;
      sq += (double)un * (double)un;
    }
    if (rows == 0) break;
  }
  if (MODE != kFwdMatvec && jb < j1) {
    if (delta > 0.0) {
      const V ub = (V)delta * (bt * ts) - cu * bub;
      u_bot[jb] = ub;
      sq += (double)ub * (double)ub;
    }
    if (pend) {
      y[jb] = by + cy * bw;
      w[jb] = bv * ts - cw * bw;
    }
  }
  const double bs = block_sum_t<kLxT>(sq);
  if (threadIdx.x == 0) beta_part[blockIdx.x] = bs;
}

// A x in sliced ELL (SELL-64) with x resident in LDS.  Slice s holds rows
// [64 s, 64 s + 64) padded to the slice's longest row (width w_s), column-major
// inside the slice: entry q of row 64 s + l at off_s + 64 q + l (padding: column
// 0, value 0).  One wave per slice, one lane per row: the value and column
// loads are fully coalesced and need only (off_s, w_s).  When every slice has
// one width uw (uw > 0) the offsets are 64 uw s, and a workgroup's first
// slice loads go out before the copy of x into LDS (one batch of 16-byte
// loads): a single dependent global round trip before the sums.  Otherwise
// (uw = 0) the slice bounds are loaded first.  Sums run in entry order (the
// CSR row order).
template <class TA, class V, int MODE>
__global__ void __launch_bounds__(kLxT)
    k_fwd_sell_lx(const int* __restrict__ soff, const int* __restrict__ swid, int nslices, int spw, int uw,
                  const int* __restrict__ sci, const TA* __restrict__ sval, long long m, long long n, const V* tin,
                  V* u_top, V* u_bot, const V* v, V* w, V* y, const GKState* __restrict__ st_in,
                  GKState* __restrict__ st_out, const double* alpha_part, int alpha_count, double* beta_part) {
  extern __shared__ __align__(16) double lx_raw[];
  V* xs = (V*)lx_raw;
  __shared__ double red[kLxT / kWave];
  GKState s = *st_in;
  const double delta = st_in->delta;
  ShareT<kLxT, 2> share;
  share.load(MODE == kFwdPlain ? alpha_part : nullptr, alpha_count);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x % kWave;
  const int sl0 = blockIdx.x * spw;
  const int sl1 = min(nslices, sl0 + spw);
  // first slice of this wave: bounds and the row's epilogue operand
  const int sa = sl0 + wave;
  const bool has_a = sa < sl1;
  int off = 0, wid = 0;
  if (has_a) {
    if (uw > 0) {
      off = sa * kWave * uw;
      wid = uw;
    } else {
      off = soff[sa];
      wid = swid[sa];
    }
  }
  const long long ra = (long long)sa * kWave + lane;
  V uo = 0;
  if (has_a && ra < m) uo = u_top[ra];
  if (MODE != kFwdMatvec && s.stop) {
    if (MODE == kFwdPlain) store_state(st_out, s);
    return;
  }
  // bottom slice [j0, j1) of the n rows
  const long long per = (n + gridDim.x - 1) / gridDim.x;
  const long long j0 = (long long)blockIdx.x * per, j1 = min(n, j0 + per);
  const long long jb = j0 + threadIdx.x;
  V bt = 0, bub = 0, bv = 0, bw = 0, by = 0;
  if (MODE != kFwdMatvec && jb < j1) {
    bt = tin[jb];
    bub = u_bot[jb];
    if (MODE == kFwdPlain) {
      bv = v[jb];
      bw = w[jb];
      by = y[jb];
    }
  }
  // values and columns of the first slice
  int cidx[kLxChunk];
  TA vv[kLxChunk];
#pragma unroll
  for (int q = 0; q < kLxChunk; ++q) {
    const bool in = q < wid;
    const long long e = (long long)off + (long long)(in ? q : 0) * kWave + lane;
    cidx[q] = in ? sci[e] : 0;
    vv[q] = in ? sval[e] : (TA)0;
  }
  // x -> LDS while the slice and bottom loads above are in flight
  x_to_lds(tin, n, xs);
  publish(share, red);
  __syncthreads();
  V ts, cu, cy = 0, cw = 0;
  bool pend = false;
  if (MODE == kFwdPlain) {
    scalar_step(s, sqrt(settled<kLxT>(red)));
    store_state(st_out, s);
    if (s.stop) {
      if (jb < j1 && s.pending) y[jb] = by + (V)s.coef_y * bw;
      return;
    }
  }
  ts = (V)(1.0 / s.alpha);
  cu = (V)(s.alpha / s.beta);
  pend = (MODE == kFwdPlain) && s.pending;
  cy = (V)s.coef_y;
  cw = (V)s.coef_w;
  double sq = 0.0;
  for (int sl = sa; sl < sl1; sl += kLxT / kWave) {
    const long long r = (long long)sl * kWave + lane;
    if (sl != sa) {
      if (uw > 0) {
        off = sl * kWave * uw;
        wid = uw;
      } else {
        off = soff[sl];
        wid = swid[sl];
      }
      uo = r < m ? u_top[r] : (V)0;
#pragma unroll
      for (int q = 0; q < kLxChunk; ++q) {
        const bool in = q < wid;
        const long long e = (long long)off + (long long)(in ? q : 0) * kWave + lane;
        cidx[q] = in ? sci[e] : 0;
        vv[q] = in ? sval[e] : (TA)0;
      }
    }
    V acc = 0;
#pragma unroll
    for (int q = 0; q < kLxChunk; ++q) acc += (V)vv[q] * xs[cidx[q]];
    for (int q = kLxChunk; q < wid; ++q) {
      const long long e = (long long)off + (long long)q * kWave + lane;
      acc += (V)sval[e] * xs[sci[e]];
    }
    if (r < m) {
      const V un = acc * ts - cu * uo;
      u_top[r] = un;
      sq += (double)un * (double)un;
    }
  }
  if (MODE != kFwdMatvec && jb < j1) {
    if (delta > 0.0) {
      const V ub = (V)delta * (bt * ts) - cu * bub;
      u_bot[jb] = ub;
      sq += (double)ub * (double)ub;
    }
    if (pend) {
      y[jb] = by + cy * bw;
      w[jb] = bv * ts - cw * bw;
    }
  }
  const double bs = block_sum_t<kLxT>(sq);
  if (threadIdx.x == 0) beta_part[blockIdx.x] = bs;
}

// Dense row-major A: one wave per row (grid-stride).
template <class TA, class V, int MODE>
__global__ void __launch_bounds__(kBlock)
    k_fwd_dense(const TA* __restrict__ A, long long m, long long n, long long ld, const V* tin, V* u_top, V* u_bot,
                const V* v, V* w, V* y, const GKState* __restrict__ st_in, GKState* __restrict__ st_out,
                const double* alpha_part, int alpha_count, double* beta_part, int row_blocks) {
  GKState s = *st_in;
  Share share;
  share.load(MODE == kFwdPlain ? alpha_part : nullptr, alpha_count);
  if (MODE != kFwdMatvec && s.stop) {
    if (MODE == kFwdPlain) store_state(st_out, s);
    return;
  }
  double sq = 0.0;
  if ((int)blockIdx.x < row_blocks) {
    __shared__ double red[kBlock / kWave];
    publish(share, red);
    __syncthreads();
    if (MODE == kFwdPlain) {
      scalar_step(s, sqrt(settled(red)));
      store_state(st_out, s);
      if (s.stop) return;
    }
    const V ts = (V)(1.0 / s.alpha), cu = (V)(s.alpha / s.beta);
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
    const long long stride = (long long)(gridDim.x - row_blocks) * kBlock;
    sq = fwd_bottom<V, MODE>(n, tin, u_bot, v, w, y, s, st_out, share,
                             (long long)(blockIdx.x - row_blocks) * kBlock + threadIdx.x, stride);
    if (MODE == kFwdPlain && s.stop) return;
  }
  const double bs = block_sum(sq);
  if (threadIdx.x == 0) beta_part[blockIdx.x] = bs;
}

// ---------------------------------------------------------------- backward kernels
// beta from the forward (or residual) partials (slot 0 -> slot 1), unless
// beta_part is null (then the state's beta is kept); g = (A^T u_top +
// delta u_bot) / beta.  PLAIN: v_raw <- g - (beta/alpha) v_raw (g at the
// phase start); otherwise g is stored for P^{-T}.  Partials of the produced
// vector's squared norm; zero partials when beta = 0 (exact solution: the
// next alpha is 0 and the scalar step stops).
template <class V, bool PLAIN>
__device__ __forceinline__ double bwd_epilogue(long long j, V dot, V ubj, V vj, V* v, V* g, double delta, V ib, V cv,
                                               int init) {
  V gj = dot * ib;
  if (delta > 0.0) gj += (V)delta * ubj * ib;
  if (PLAIN) {
    const V vn = init ? gj : gj - cv * vj;
    v[j] = vn;
    return (double)vn * (double)vn;
  } else {
    g[j] = gj;
    return (double)gj * (double)gj;
  }
}

struct BwdScal {
  double ib, cv;
  bool zero;
};

// Finishes beta from `total` (or keeps the state's beta); workgroup 0
// stores the advanced state.
__device__ __forceinline__ bool bwd_settle(const GKState* __restrict__ st_in, GKState* __restrict__ st_out,
                                          bool finish_beta, double total, BwdScal& k) {
  double beta = st_in->beta;
  int stop = 0;
  if (finish_beta) {
    beta = sqrt(total);
    stop = !(beta == beta) || isinf(beta) || (beta == 0.0 && st_in->init);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    GKState o = *st_in;
    if (finish_beta) beta_step(o, total);
    *st_out = o;
  }
  if (stop) return false;
  if (beta == 0.0) {
    k.zero = true;
    return false;
  }
  k.ib = 1.0 / beta;
  k.cv = beta / st_in->alpha;
  return true;
}

// KS: producer partials held per thread (1 when the forward grid is at most
// kBlock workgroups, which keeps the kernel at seven workgroups per CU).
template <class TA, class V, bool PLAIN, bool BOT, int KS>
__global__ void __launch_bounds__(kBlock)
    k_bwd_csr(const RowBlk* __restrict__ trbk, const int* __restrict__ tp, const int* __restrict__ ti,
              const TA* __restrict__ tv, const V* u_top, const V* u_bot, V* v, V* g,
              const GKState* __restrict__ st_in, GKState* __restrict__ st_out, const double* beta_part,
              int beta_count, double* alpha_part) {
  const RowBlk ra = trbk[blockIdx.x], rb = trbk[blockIdx.x + 1];
  const int stop0 = st_in->stop, init = st_in->init;
  const double delta = st_in->delta;
  ShareT<kBlock, KS> share;
  share.load(beta_part, beta_count);
  if (stop0) {
    store_state(st_out, *st_in);
    return;
  }
  BwdScal k{0.0, 0.0, false};
  double sq = 0.0;
  const bool ran = csr_stream<V>(
      ra, rb, tp, ti, tv, u_top, share,
      [&](int j, V& q0, V& q1) {
        q0 = BOT ? u_bot[j] : (V)0;
        q1 = PLAIN ? v[j] : (V)0;
      },
      [&](double total) { return bwd_settle(st_in, st_out, beta_part != nullptr, total, k); },
      [&](int j, V dot, V q0, V q1) {
        sq += bwd_epilogue<V, PLAIN>(j, dot, q0, q1, v, g, delta, (V)k.ib, (V)k.cv, init);
      });
  if (!ran) {
    if (k.zero && threadIdx.x == 0) alpha_part[blockIdx.x] = 0.0;
    return;
  }
  const double bs = block_sum(sq);
  if (threadIdx.x == 0) alpha_part[blockIdx.x] = bs;
}

// Dense A^T u: partial sums over row chunks (threads along columns, coalesced).
template <class TA, class V>
__global__ void __launch_bounds__(kBlock)
    k_bwd_dense_part(const TA* __restrict__ A, long long m, long long n, long long ld, const V* __restrict__ u_top,
                     double* part, long long rpc, const GKState* __restrict__ sl) {
  if (sl && sl->stop) return;
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
                    const GKState* __restrict__ st_in, GKState* __restrict__ st_out, const double* beta_part,
                    int beta_count, double* alpha_part) {
  __shared__ double red[kBlock / kWave];
  Share share;
  share.load(beta_part, beta_count);
  if (st_in->stop) {
    store_state(st_out, *st_in);
    return;
  }
  BwdScal k{0.0, 0.0, false};
  publish(share, red);
  __syncthreads();
  if (!bwd_settle(st_in, st_out, beta_part != nullptr, settled(red), k)) {
    if (k.zero && threadIdx.x == 0) alpha_part[blockIdx.x] = 0.0;
    return;
  }
  const double delta = st_in->delta;
  const int init = st_in->init;
  double sq = 0.0;
  for (long long j = (long long)blockIdx.x * kBlock + threadIdx.x; j < n; j += (long long)gridDim.x * kBlock) {
    double acc = 0.0;
    for (int c = 0; c < chunks; ++c) acc += part[(long long)c * n + j];
    const V ubj = delta > 0.0 ? u_bot[j] : (V)0;
    const V vj = (PLAIN && !init) ? v[j] : (V)0;
    sq += bwd_epilogue<V, PLAIN>(j, (V)acc, ubj, vj, v, g, delta, (V)k.ib, (V)k.cv, init);
  }
  const double bs = block_sum(sq);
  if (threadIdx.x == 0) alpha_part[blockIdx.x] = bs;
}

// ---------------------------------------------------------------- P^{-1} coefficients
// Both forms apply P^{-1} z = z + V (d .* (V^T z)) with V = Q_R V_M.
// Explicit (dense A): V row-major n x ell; c = d .* (V^T z) by chunk partials
// and an ordered chunk sum.  Implicit (CSR A): Q_R = R^T T_R^{-1} with
// R = A(I,:), so V = R^T K, K = T_R^{-1} V_M (ell x ell); c1 = R z,
// w = d .* (K^T c1), c = K w, and the consumer adds R^T c.
template <class V>
__global__ void __launch_bounds__(kBlock)
    k_pa_part(const double* __restrict__ Vh, long long n, int ell, long long ldv, const V* __restrict__ z,
              double* part, long long rpc, const GKState* sl) {
  if (sl && sl->stop) return;
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= ell) return;
  const long long i0 = (long long)blockIdx.y * rpc;
  const long long i1 = min(n, i0 + rpc);
  double acc = 0.0;
  for (long long i = i0; i < i1; ++i) acc += Vh[i * ldv + k] * (double)z[i];
  part[(long long)blockIdx.y * ell + k] = acc;
}

// 64 columns per workgroup, the four waves take chunks q, q + 4, ... and are
// summed in order.
__global__ void __launch_bounds__(kBlock)
    k_pa_red(const double* __restrict__ part, int chunks, int ell, const double* __restrict__ d, double* c,
             const GKState* sl) {
  __shared__ double acc4[kBlock / kWave][kWave];
  if (sl && sl->stop) return;
  const int col = blockIdx.x * kWave + threadIdx.x % kWave, q = threadIdx.x / kWave;
  double acc = 0.0;
  if (col < ell) {
#pragma unroll 4
    for (int ch = q; ch < chunks; ch += kBlock / kWave) acc += part[(long long)ch * ell + col];
  }
  acc4[q][threadIdx.x % kWave] = acc;
  __syncthreads();
  if (q == 0 && col < ell) {
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kBlock / kWave; ++i) t += acc4[i][threadIdx.x];
    c[col] = d ? d[col] * t : t;
  }
}

// c1[k] = A(I[k], :) . z  (groups of 16 lanes per row).
template <class TA, class V>
__global__ void __launch_bounds__(kBlock)
    k_pr_rz(const int* __restrict__ rp, const int* __restrict__ ci, const TA* __restrict__ val,
            const int* __restrict__ I, int ell, const V* __restrict__ z, double* c1, const GKState* sl) {
  constexpr int G = 16;
  if (sl && sl->stop) return;
  const int k = blockIdx.x * (kBlock / G) + threadIdx.x / G, lane = threadIdx.x % G;
  if (k >= ell) return;  // whole groups leave together
  const int r = I[k];
  double acc = 0.0;
  for (int e = rp[r] + lane; e < rp[r + 1]; e += G) acc += (double)val[e] * (double)z[ci[e]];
  for (int off = G >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
  if (lane == 0) c1[k] = acc;
}

// y = diag(dscale) M x (dscale may be null), M row-major ell x ell; one wave per row.
__global__ void __launch_bounds__(kBlock)
    k_pr_gemv(const double* __restrict__ M, int ell, const double* __restrict__ x, const double* __restrict__ dscale,
              double* y, const GKState* sl) {
  if (sl && sl->stop) return;
  const int row = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave, lane = threadIdx.x % kWave;
  if (row >= ell) return;
  const double* a = M + (long long)row * ell;
  double acc = 0.0;
#pragma unroll 4
  for (int k = lane; k < ell; k += kWave) acc += a[k] * x[k];
  acc = wave_sum(acc);
  if (lane == 0) y[row] = dscale ? dscale[row] * acc : acc;
}

// (P^{-1} - I) z at row j: the explicit row dot V(j,:) . c (one wave) or the
// implicit R^T row (one thread).
__device__ __forceinline__ double vrow_dot(const double* __restrict__ Vh, long long ldv, int ell,
                                           const double* __restrict__ c, long long i, int lane) {
  double acc = 0.0;
  const double* r = Vh + i * ldv;
  for (int k = lane; k < ell; k += kWave) acc += r[k] * c[k];
  return wave_sum(acc);
}

__device__ __forceinline__ double rt_dot(const int* __restrict__ tp, const int* __restrict__ ti,
                                         const double* __restrict__ tv, const double* __restrict__ c, long long j) {
  double acc = 0.0;
  for (int e = tp[j]; e < tp[j + 1]; ++e) acc += tv[e] * c[ti[e]];
  return acc;
}

// Row loop of the P-apply consumers: one wave per row (explicit) or one
// thread per row (implicit); f(j, dot) runs in one lane per row.
template <class F>
__device__ __forceinline__ void prec_rows(const PrecDesc& P, long long n, F&& f) {
  if (!P.implicit) {
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    constexpr int rpb = kBlock / kWave;
    for (long long i = (long long)blockIdx.x * rpb + wv; i < n; i += (long long)gridDim.x * rpb) {
      const double dot = vrow_dot(P.V, P.ldv, P.ell, P.c, i, lane);
      if (lane == 0) f(i, dot);
    }
  } else {
    for (long long j = (long long)blockIdx.x * kBlock + threadIdx.x; j < n; j += (long long)gridDim.x * kBlock)
      f(j, rt_dot(P.rt_ptr, P.rt_idx, P.rt_val, P.c, j));
  }
}

// First kernel of a preconditioned iteration: finishes alpha (partials of
// the previous P^{-T} kernel; slot 1 -> slot 0), takes the scalar step,
// applies the y/w update and forms t = P^{-1} v_raw = v_raw + (P^{-1} - I) v_raw.
template <class V>
__global__ void __launch_bounds__(kBlock)
    k_pa_fwd(const PrecDesc P, long long n, const V* v, V* t, V* w, V* y, const GKState* __restrict__ st_in,
             GKState* __restrict__ st_out, const double* alpha_part, int alpha_count) {
  __shared__ double red[kBlock / kWave];
  GKState s = *st_in;
  Share share;
  share.load(alpha_part, alpha_count);
  if (s.stop) {
    store_state(st_out, s);
    return;
  }
  publish(share, red);
  __syncthreads();
  scalar_step(s, sqrt(settled(red)));
  store_state(st_out, s);
  if (s.stop) {
    final_y<V>(n, y, w, s, (long long)blockIdx.x * kBlock + threadIdx.x, (long long)gridDim.x * kBlock);
    return;
  }
  const bool pend = s.pending;
  const double cy = s.coef_y, cw = s.coef_w, ia = 1.0 / s.alpha;
  prec_rows(P, n, [&](long long i, double dot) {
    const V vi = v[i];
    t[i] = (V)((double)vi + dot);
    if (pend) {
      const V wi = w[i];
      y[i] += (V)cy * wi;
      w[i] = (V)((double)vi * ia) - (V)cw * wi;
    }
  });
}

// v_raw <- P^{-1} g - (beta/alpha) v_raw  (P^{-1} g at the phase start);
// partials of ||v_raw||^2 (slot 1 holds beta).
template <class V>
__global__ void __launch_bounds__(kBlock)
    k_pa_bwd(const PrecDesc P, long long n, const V* g, V* v, const GKState* __restrict__ sl, double* alpha_part) {
  if (sl->stop) return;
  const int init = sl->init;
  const double cv = sl->beta / sl->alpha;
  double sq = 0.0;
  prec_rows(P, n, [&](long long i, double dot) {
    const double pg = (double)g[i] + dot;
    const V vn = init ? (V)pg : (V)(pg - cv * (double)v[i]);
    v[i] = vn;
    sq += (double)vn * (double)vn;
  });
  const double bs = block_sum(sq);
  if (threadIdx.x == 0) alpha_part[blockIdx.x] = bs;
}

// x += P^{-1} y  (x in FP64).
template <class V>
__global__ void __launch_bounds__(kBlock) k_pa_x(const PrecDesc P, long long n, const V* y, double* x) {
  prec_rows(P, n, [&](long long i, double dot) { x[i] += (double)y[i] + dot; });
}

// ---------------------------------------------------------------- phase start / end
// r_top = b - A x (FP64, values widened), r_bot = bot_scale b_bot - delta x;
// partials of ||r||^2.
template <class TA, class RV>
__global__ void __launch_bounds__(kBlock)
    k_resid_csr(const RowBlk* __restrict__ rbk, const int* __restrict__ rp, const int* __restrict__ ci,
                const TA* __restrict__ val, long long m, long long n, const double* __restrict__ b,
                const double* b_bot, double bot_scale, const double* x, int x_zero, RV* r_top, RV* r_bot,
                const GKState* __restrict__ sl, double* beta_part, int row_blocks) {
  const double delta = sl->delta;
  double sq = 0.0;
  if ((int)blockIdx.x < row_blocks) {
    const RowBlk a = rbk[blockIdx.x], bb = rbk[blockIdx.x + 1];
    if (x_zero) {
      for (int r = a.r0 + threadIdx.x; r < bb.r0; r += kBlock) {
        const double rr = b ? b[r] : 0.0;
        r_top[r] = (RV)rr;
        sq += rr * rr;
      }
    } else {
      Share none;
      none.load(nullptr, 0);
      csr_stream<double>(
          a, bb, rp, ci, val, x, none,
          [&](int r, double& q0, double& q1) {
            q0 = b ? b[r] : 0.0;
            q1 = 0.0;
          },
          [&](double) { return true; },
          [&](int r, double dot, double q0, double) {
            const double rr = q0 - dot;
            r_top[r] = (RV)rr;
            sq += rr * rr;
          });
    }
  } else if (delta > 0.0) {
    const int nb = gridDim.x - row_blocks;
    for (long long j = (long long)(blockIdx.x - row_blocks) * kBlock + threadIdx.x; j < n; j += (long long)nb * kBlock) {
      double r = x_zero ? 0.0 : -delta * x[j];
      if (b_bot) r += bot_scale * b_bot[j];
      r_bot[j] = (RV)r;
      sq += r * r;
    }
  }
  const double bs = block_sum(sq);
  if (threadIdx.x == 0) beta_part[blockIdx.x] = bs;
}

template <class TA, class RV>
__global__ void __launch_bounds__(kBlock)
    k_resid_dense(const TA* __restrict__ A, long long m, long long n, long long ld, const double* __restrict__ b,
                  const double* b_bot, double bot_scale, const double* x, int x_zero, RV* r_top, RV* r_bot,
                  const GKState* __restrict__ sl, double* beta_part, int row_blocks) {
  const double delta = sl->delta;
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
        r_top[row] = (RV)r;
        sq += r * r;
      }
    }
  } else if (delta > 0.0) {
    const int nb = gridDim.x - row_blocks;
    for (long long j = (long long)(blockIdx.x - row_blocks) * kBlock + threadIdx.x; j < n; j += (long long)nb * kBlock) {
      double r = x_zero ? 0.0 : -delta * x[j];
      if (b_bot) r += bot_scale * b_bot[j];
      r_bot[j] = (RV)r;
      sq += r * r;
    }
  }
  const double bs = block_sum(sq);
  if (threadIdx.x == 0) beta_part[blockIdx.x] = bs;
}

// One workgroup: finish a reduction into slot 0.  mode 0: alpha and the
// scalar step (slot 1 -> slot 0); mode 1: beta (slot 0 -> slot 0).
__global__ void __launch_bounds__(kBlock) k_consume(GKState* st, const double* part, int count, int mode) {
  __shared__ double red[kBlock / kWave];
  GKState s = st[mode == 0 ? 1 : 0];
  Share share;
  share.load(part, count);
  publish(share, red);
  __syncthreads();
  if (!s.stop) {
    if (mode == 0)
      scalar_step(s, sqrt(settled(red)));
    else
      beta_step(s, settled(red));
  }
  __syncthreads();
  store_state(&st[0], s);
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
static unsigned clamp_grid(long long want, long long cap = kMaxGrid) {
  if (want < 1) return 1;
  return (unsigned)(want > cap ? cap : want);
}
static unsigned nbottom(long long n) { return clamp_grid(ceil_div(n, kBlock), 64); }
static unsigned fwd_row_blocks(const OpDesc& A) {
  if (A.csr) return (unsigned)stream_blocks(A.nnz, A.stream_t);
  return clamp_grid((A.m + 3) / 4);
}
static unsigned bwd_grid(const OpDesc& A) {
  if (A.csr) return (unsigned)stream_blocks(A.nnz, A.stream_t);
  return clamp_grid(ceil_div(A.n, kBlock), 1024);
}
static unsigned prec_grid(const PrecDesc& P, long long n) {
  return P.implicit ? clamp_grid(ceil_div(n, kBlock), kRowsMaxGrid) : clamp_grid((n + 3) / 4, kRowsMaxGrid);
}

// Launch; with events, through the dispatch-timed launch (the events take the
// kernel's own start and end timestamps, as a kernel trace does).
template <class F, class... Args>
static void launch_kx(F kern, dim3 g, dim3 b, unsigned shm, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                      Args... args) {
  if (e0 || e1)
    hipExtLaunchKernelGGL(kern, g, b, shm, s, e0, e1, 0, args...);
  else
    hipLaunchKernelGGL(kern, g, b, shm, s, args...);
}
template <class F, class... Args>
static void launch_k(F kern, dim3 g, hipStream_t s, hipEvent_t e0, hipEvent_t e1, Args... args) {
  launch_kx(kern, g, dim3(kBlock), 0u, s, e0, e1, args...);
}

// Dynamic LDS of the LDS-resident forward kernels (kLxMaxBytes: the x copy).
template <class TA, class V>
static void lx_attr() {
  (void)hipFuncSetAttribute((const void*)k_fwd_csr_lx<TA, V, kFwdPlain>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)kLxMaxBytes);
  (void)hipFuncSetAttribute((const void*)k_fwd_csr_lx<TA, V, kFwdPre>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)kLxMaxBytes);
  (void)hipFuncSetAttribute((const void*)k_fwd_csr_lx<TA, V, kFwdMatvec>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLxMaxBytes);
  (void)hipFuncSetAttribute((const void*)k_fwd_sell_lx<TA, V, kFwdPlain>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)kLxMaxBytes);
  (void)hipFuncSetAttribute((const void*)k_fwd_sell_lx<TA, V, kFwdPre>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)kLxMaxBytes);
  (void)hipFuncSetAttribute((const void*)k_fwd_sell_lx<TA, V, kFwdMatvec>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLxMaxBytes);
}

// ---------------------------------------------------------------- SELL-64 copy of a CSR matrix
__global__ void k_sell_widths(const int* rp, long long m, int* wid) {
  const long long r = (long long)blockIdx.x * kBlock + threadIdx.x;
  int len = r < m ? rp[r + 1] - rp[r] : 0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) len = max(len, __shfl_xor(len, o, kWave));
  if (threadIdx.x % kWave == 0 && r - threadIdx.x % kWave < m) wid[r / kWave] = len;
}

template <class TA>
__global__ void k_sell_fill(const int* rp, const int* ci, const TA* val, long long m, const int* off, const int* wid,
                            int* sci, TA* sval) {
  const long long r = (long long)blockIdx.x * kBlock + threadIdx.x;
  const long long sl = r / kWave;
  const int lane = (int)(r % kWave);
  if (sl >= (m + kWave - 1) / kWave) return;
  const int b = r < m ? rp[r] : 0, len = r < m ? rp[r + 1] - b : 0;
  const long long base = off[sl];
  for (int q = 0; q < wid[sl]; ++q) {
    const long long e = base + (long long)q * kWave + lane;
    sci[e] = q < len ? ci[b + q] : 0;
    sval[e] = q < len ? val[b + q] : (TA)0;
  }
}

// Widths of the SELL-64 slices of (rp, m) into wid (host vector); returns the
// padded entry count.
long long sell_widths(const int* rp, long long m, int* wid_dev, std::vector<int>& wid_host, hipStream_t s) {
  const long long ns = (m + kWave - 1) / kWave;
  hipLaunchKernelGGL(k_sell_widths, dim3(ceil_div(ns * kWave, kBlock)), dim3(kBlock), 0, s, rp, m, wid_dev);
  wid_host.resize(ns);
  APL_HIP(hipMemcpyAsync(wid_host.data(), wid_dev, sizeof(int) * ns, hipMemcpyDeviceToHost, s));
  APL_HIP(hipStreamSynchronize(s));
  long long total = 0;
  for (int w : wid_host) total += (long long)w * kWave;
  return total;
}

template <class TA>
void sell_fill(const int* rp, const int* ci, const TA* val, long long m, const int* off_dev, const int* wid_dev,
               int* sci, TA* sval, hipStream_t s) {
  const long long ns = (m + kWave - 1) / kWave;
  hipLaunchKernelGGL(k_sell_fill<TA>, dim3(ceil_div(ns * kWave, kBlock)), dim3(kBlock), 0, s, rp, ci, val, m, off_dev,
                     wid_dev, sci, sval);
}
template void sell_fill<double>(const int*, const int*, const double*, long long, const int*, const int*, int*,
                                double*, hipStream_t);
template void sell_fill<float>(const int*, const int*, const float*, long long, const int*, const int*, int*, float*,
                               hipStream_t);

// Once per process: kernel attributes (the LDS-resident kernel's dynamic LDS).
void gk_prepare() {
  static const bool done = []() {
    lx_attr<double, double>();
    lx_attr<float, double>();
    lx_attr<double, float>();
    lx_attr<float, float>();
    return true;
  }();
  (void)done;
}

static int device_cus() {
  static const int cus = []() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
      v = 256;
    return v;
  }();
  return cus;
}

// Row blocks of the LDS-resident forward kernel: one per CU, balanced by non-zeros.
int lx_stream_t(long long nnz) { return (int)std::max<long long>(1, (nnz + device_cus() - 1) / device_cus()); }

// SELL-64 launch: about one workgroup per CU, and enough workgroups that each
// owns at most kLxT of the n bottom rows.
void sell_layout(long long nslices, long long n, int* spw, int* grid) {
  const long long per = std::max<long long>(1, (nslices + device_cus() - 1) / device_cus());
  *spw = (int)per;
  *grid = (int)std::max<long long>(std::max<long long>(1, (nslices + per - 1) / per), (n + kLxT - 1) / kLxT);
}

template <class V, int MODE>
static void launch_fwd(const OpDesc& A, const V* tin, GKVecs<V> vec, GKState* st, GKWork& wk, hipStream_t s,
                       hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  const unsigned rb = fwd_row_blocks(A);
  const unsigned grid = rb + nbottom(A.n);
  const int ac = (int)wk.alpha_count;
  const GKState* sin = st + (MODE == kFwdPlain ? 1 : 0);
  GKState* sout = (MODE == kFwdPlain) ? st : nullptr;
  if (A.csr && A.sell_off && A.nnz >= kLxMinNnz && A.n * (long long)sizeof(V) <= kLxMaxBytes) {
    const unsigned lg = (unsigned)A.sell_grid;
    const unsigned shm = (unsigned)(A.n * sizeof(V));
    if (A.f64)
      launch_kx(k_fwd_sell_lx<double, V, MODE>, dim3(lg), dim3(kLxT), shm, s, e0, e1, A.sell_off, A.sell_w,
                A.sell_slices, A.sell_spw, A.sell_uw, A.sell_ci, (const double*)A.sell_val, A.m, A.n, tin, vec.u_top, vec.u_bot,
                (const V*)vec.v, vec.w, vec.y, sin, sout, (const double*)wk.alpha_part, ac, wk.beta_part);
    else
      launch_kx(k_fwd_sell_lx<float, V, MODE>, dim3(lg), dim3(kLxT), shm, s, e0, e1, A.sell_off, A.sell_w,
                A.sell_slices, A.sell_spw, A.sell_uw, A.sell_ci, (const float*)A.sell_val, A.m, A.n, tin, vec.u_top, vec.u_bot,
                (const V*)vec.v, vec.w, vec.y, sin, sout, (const double*)wk.alpha_part, ac, wk.beta_part);
    wk.beta_count = lg;
    return;
  }
  if (A.csr && A.lx_rb && A.nnz >= kLxMinNnz && A.n * (long long)sizeof(V) <= kLxMaxBytes) {
    const RowBlk* lrb = (const RowBlk*)A.lx_rb;
    const unsigned lg = (unsigned)A.lx_grid;
    const unsigned shm = (unsigned)(A.n * sizeof(V));
    if (A.f64)
      launch_kx(k_fwd_csr_lx<double, V, MODE>, dim3(lg), dim3(kLxT), shm, s, e0, e1, lrb, A.row_ptr, A.col_idx,
                (const double*)A.val, A.n, tin, vec.u_top, vec.u_bot, (const V*)vec.v, vec.w, vec.y, sin, sout,
                (const double*)wk.alpha_part, ac, wk.beta_part);
    else
      launch_kx(k_fwd_csr_lx<float, V, MODE>, dim3(lg), dim3(kLxT), shm, s, e0, e1, lrb, A.row_ptr, A.col_idx,
                (const float*)A.val, A.n, tin, vec.u_top, vec.u_bot, (const V*)vec.v, vec.w, vec.y, sin, sout,
                (const double*)wk.alpha_part, ac, wk.beta_part);
    wk.beta_count = lg;
    return;
  }
  if (A.csr) {
    const RowBlk* rbk = (const RowBlk*)A.rb;
    if (A.f64)
      launch_k(k_fwd_csr<double, V, MODE>, dim3(grid), s, e0, e1, rbk, A.row_ptr, A.col_idx, (const double*)A.val,
               A.n, tin, vec.u_top, vec.u_bot, (const V*)vec.v, vec.w, vec.y, sin, sout,
               (const double*)wk.alpha_part, ac, wk.beta_part, (int)rb);
    else
      launch_k(k_fwd_csr<float, V, MODE>, dim3(grid), s, e0, e1, rbk, A.row_ptr, A.col_idx, (const float*)A.val,
               A.n, tin, vec.u_top, vec.u_bot, (const V*)vec.v, vec.w, vec.y, sin, sout,
               (const double*)wk.alpha_part, ac, wk.beta_part, (int)rb);
  } else {
    if (A.f64)
      launch_k(k_fwd_dense<double, V, MODE>, dim3(grid), s, e0, e1, (const double*)A.val, A.m, A.n, A.ld, tin,
               vec.u_top, vec.u_bot, (const V*)vec.v, vec.w, vec.y, sin, sout, (const double*)wk.alpha_part, ac,
               wk.beta_part, (int)rb);
    else
      launch_k(k_fwd_dense<float, V, MODE>, dim3(grid), s, e0, e1, (const float*)A.val, A.m, A.n, A.ld, tin,
               vec.u_top, vec.u_bot, (const V*)vec.v, vec.w, vec.y, sin, sout, (const double*)wk.alpha_part, ac,
               wk.beta_part, (int)rb);
  }
  wk.beta_count = grid;
}

// beta_from_part: finish beta from wk.beta_part (else the state's beta is kept).
template <class V, bool PLAIN>
static void launch_bwd(const OpDesc& A, const V* u_top, const V* u_bot, V* v, V* g, GKState* st, GKWork& wk,
                       bool beta_from_part, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  const double* bp = beta_from_part ? wk.beta_part : nullptr;
  const int bc = (int)wk.beta_count;
  const unsigned grid = bwd_grid(A);
  if (A.csr) {
    const RowBlk* trbk = (const RowBlk*)A.t_rb;
    const GKState* sin = st;
    GKState* sout = st + 1;
    auto go = [&](auto kern, const auto* tv) {
      launch_k(kern, dim3(grid), s, e0, e1, trbk, A.t_ptr, A.t_idx, tv, u_top, u_bot, v, g, sin, sout, bp, bc,
               wk.alpha_part);
    };
    const bool one = !bp || bc <= kBlock;
    if (A.f64) {
      const double* tv = (const double*)A.t_val;
      if (u_bot)
        one ? go(k_bwd_csr<double, V, PLAIN, true, 1>, tv) : go(k_bwd_csr<double, V, PLAIN, true, kShare>, tv);
      else
        one ? go(k_bwd_csr<double, V, PLAIN, false, 1>, tv) : go(k_bwd_csr<double, V, PLAIN, false, kShare>, tv);
    } else {
      const float* tv = (const float*)A.t_val;
      if (u_bot)
        one ? go(k_bwd_csr<float, V, PLAIN, true, 1>, tv) : go(k_bwd_csr<float, V, PLAIN, true, kShare>, tv);
      else
        one ? go(k_bwd_csr<float, V, PLAIN, false, 1>, tv) : go(k_bwd_csr<float, V, PLAIN, false, kShare>, tv);
    }
  } else {
    const long long rpc = (A.m + A.chunks - 1) / A.chunks;
    dim3 g1(ceil_div(A.n, kBlock), A.chunks);
    if (A.f64)
      launch_k(k_bwd_dense_part<double, V>, g1, s, e0, nullptr, (const double*)A.val, A.m, A.n, A.ld, u_top, A.part,
               rpc, (const GKState*)st);
    else
      launch_k(k_bwd_dense_part<float, V>, g1, s, e0, nullptr, (const float*)A.val, A.m, A.n, A.ld, u_top, A.part,
               rpc, (const GKState*)st);
    launch_k(k_bwd_dense_red<V, PLAIN>, dim3(grid), s, nullptr, e1, (const double*)A.part, A.chunks, A.n, u_bot, v,
             g, (const GKState*)st, st + 1, bp, bc, wk.alpha_part);
  }
  wk.alpha_count = grid;
}

// P.c <- the coefficients of (P^{-1} - I) z, or of (P^{-T} - I) z when trans
// (stop check on slot sl, or none).
template <class V>
static void launch_pcoef(const OpDesc& A, const PrecDesc& P, long long n, const V* z, const GKState* sl, bool trans,
                         hipStream_t s) {
  const double* Mid = (trans && P.M2t) ? P.M2t : P.M2;
  if (!P.implicit) {
    const long long rpc = (n + P.chunks - 1) / P.chunks;
    hipLaunchKernelGGL((k_pa_part<V>), dim3(ceil_div(P.ell, kBlock), P.chunks), dim3(kBlock), 0, s, P.V, n, P.ell,
                       P.ldv, z, P.part, rpc, sl);
    if (!Mid) {
      hipLaunchKernelGGL(k_pa_red, dim3(ceil_div(P.ell, kWave)), dim3(kBlock), 0, s, P.part, P.chunks, P.ell, P.d,
                         P.c, sl);
      return;
    }
    hipLaunchKernelGGL(k_pa_red, dim3(ceil_div(P.ell, kWave)), dim3(kBlock), 0, s, P.part, P.chunks, P.ell,
                       (const double*)nullptr, P.c2, sl);
    hipLaunchKernelGGL(k_pr_gemv, dim3(ceil_div(P.ell, kBlock / kWave)), dim3(kBlock), 0, s, Mid, P.ell,
                       (const double*)P.c2, (const double*)nullptr, P.c, sl);
    return;
  }
  const unsigned g1 = ceil_div(P.ell, kBlock / 16);
  if (A.f64)
    hipLaunchKernelGGL((k_pr_rz<double, V>), dim3(g1), dim3(kBlock), 0, s, A.row_ptr, A.col_idx,
                       (const double*)A.val, P.I, P.ell, z, P.c1, sl);
  else
    hipLaunchKernelGGL((k_pr_rz<float, V>), dim3(g1), dim3(kBlock), 0, s, A.row_ptr, A.col_idx,
                       (const float*)A.val, P.I, P.ell, z, P.c1, sl);
  const unsigned g2 = ceil_div(P.ell, kBlock / kWave);
  if (Mid) {
    hipLaunchKernelGGL(k_pr_gemv, dim3(g2), dim3(kBlock), 0, s, Mid, P.ell, (const double*)P.c1,
                       (const double*)nullptr, P.c, sl);
    return;
  }
  hipLaunchKernelGGL(k_pr_gemv, dim3(g2), dim3(kBlock), 0, s, P.Kt, P.ell, (const double*)P.c1, P.d, P.c2, sl);
  hipLaunchKernelGGL(k_pr_gemv, dim3(g2), dim3(kBlock), 0, s, P.Kr, P.ell, (const double*)P.c2,
                     (const double*)nullptr, P.c, sl);
}

template <class V>
void gk_iteration(const OpDesc& A, const PrecDesc* P, GKVecs<V> vec, GKState* st, GKWork& wk, hipStream_t s) {
  if (!P) {
    launch_fwd<V, kFwdPlain>(A, vec.v, vec, st, wk, s);
    launch_bwd<V, true>(A, vec.u_top, vec.u_bot, vec.v, vec.g, st, wk, true, s);
    return;
  }
  const unsigned pg = prec_grid(*P, A.n);
  launch_pcoef<V>(A, *P, A.n, vec.v, &st[1], false, s);
  hipLaunchKernelGGL((k_pa_fwd<V>), dim3(pg), dim3(kBlock), 0, s, *P, A.n, (const V*)vec.v, vec.t, vec.w, vec.y,
                     (const GKState*)(st + 1), st, (const double*)wk.alpha_part, (int)wk.alpha_count);
  launch_fwd<V, kFwdPre>(A, vec.t, vec, st, wk, s);
  launch_bwd<V, false>(A, vec.u_top, vec.u_bot, vec.v, vec.g, st, wk, true, s);
  launch_pcoef<V>(A, *P, A.n, vec.g, &st[1], true, s);
  hipLaunchKernelGGL((k_pa_bwd<V>), dim3(pg), dim3(kBlock), 0, s, *P, A.n, (const V*)vec.g, vec.v,
                     (const GKState*)(st + 1), wk.alpha_part);
  wk.alpha_count = pg;
}

template <class RV>
static void launch_resid(const OpDesc& A, const double* b, const double* b_bot, double bot_scale, const double* x,
                         RV* r_top, RV* r_bot, GKState* st, GKWork& wk, hipStream_t s) {
  const int x_zero = (x == nullptr);
  const unsigned rb = fwd_row_blocks(A);
  const unsigned grid = rb + nbottom(A.n);
  if (A.csr) {
    const RowBlk* rbk = (const RowBlk*)A.rb;
    if (A.f64)
      hipLaunchKernelGGL((k_resid_csr<double, RV>), dim3(grid), dim3(kBlock), 0, s, rbk, A.row_ptr, A.col_idx,
                         (const double*)A.val, A.m, A.n, b, b_bot, bot_scale, x, x_zero, r_top, r_bot,
                         (const GKState*)st, wk.beta_part, (int)rb);
    else
      hipLaunchKernelGGL((k_resid_csr<float, RV>), dim3(grid), dim3(kBlock), 0, s, rbk, A.row_ptr, A.col_idx,
                         (const float*)A.val, A.m, A.n, b, b_bot, bot_scale, x, x_zero, r_top, r_bot,
                         (const GKState*)st, wk.beta_part, (int)rb);
  } else {
    if (A.f64)
      hipLaunchKernelGGL((k_resid_dense<double, RV>), dim3(grid), dim3(kBlock), 0, s, (const double*)A.val, A.m, A.n,
                         A.ld, b, b_bot, bot_scale, x, x_zero, r_top, r_bot, (const GKState*)st, wk.beta_part,
                         (int)rb);
    else
      hipLaunchKernelGGL((k_resid_dense<float, RV>), dim3(grid), dim3(kBlock), 0, s, (const float*)A.val, A.m, A.n,
                         A.ld, b, b_bot, bot_scale, x, x_zero, r_top, r_bot, (const GKState*)st, wk.beta_part,
                         (int)rb);
  }
  wk.beta_count = grid;
}

template <class V>
void gk_phase_init(const OpDesc& Ares, const OpDesc& A, const PrecDesc* P, const double* b, const double* b_bot,
                   double bot_scale, const double* x, GKVecs<V> vec, GKState* st, GKWork& wk, hipStream_t s) {
  launch_resid<V>(Ares, b, b_bot, bot_scale, x, vec.u_top, vec.u_bot, st, wk, s);
  fill_zero<V>(vec.y, A.n, s);
  fill_zero<V>(vec.w, A.n, s);
  if (!P) {
    launch_bwd<V, true>(A, (const V*)vec.u_top, (const V*)vec.u_bot, vec.v, vec.g, st, wk, true, s);
  } else {
    launch_bwd<V, false>(A, (const V*)vec.u_top, (const V*)vec.u_bot, vec.v, vec.g, st, wk, true, s);
    launch_pcoef<V>(A, *P, A.n, vec.g, &st[1], true, s);
    const unsigned pg = prec_grid(*P, A.n);
    hipLaunchKernelGGL((k_pa_bwd<V>), dim3(pg), dim3(kBlock), 0, s, *P, A.n, (const V*)vec.g, vec.v,
                       (const GKState*)(st + 1), wk.alpha_part);
    wk.alpha_count = pg;
  }
}

// x += P^{-1} y.  The last y update was applied by the kernel that stopped.
template <class V>
void gk_phase_finish(const OpDesc& A, const PrecDesc* P, GKVecs<V> vec, double* x, GKState* st, hipStream_t s) {
  (void)st;
  if (!P) {
    hipLaunchKernelGGL((k_axpy_x<V>), dim3(clamp_grid(ceil_div(A.n, kBlock))), dim3(kBlock), 0, s, A.n,
                       (const V*)vec.y, x);
  } else {
    launch_pcoef<V>(A, *P, A.n, vec.y, nullptr, false, s);
    hipLaunchKernelGGL((k_pa_x<V>), dim3(prec_grid(*P, A.n)), dim3(kBlock), 0, s, *P, A.n, (const V*)vec.y, x);
  }
}

// y = P^{-1} z (trans = false) or P^{-T} z (trans = true) with the
// coefficient kernels of the LSQR iteration and the row pass of the phase end.
void gk_precond_apply(const OpDesc& A, const PrecDesc& P, bool trans, const double* z, double* y, hipStream_t s) {
  fill_zero<double>(y, A.n, s);
  launch_pcoef<double>(A, P, A.n, z, nullptr, trans, s);
  hipLaunchKernelGGL((k_pa_x<double>), dim3(prec_grid(P, A.n)), dim3(kBlock), 0, s, P, A.n, z, y);
}

template void gk_iteration<double>(const OpDesc&, const PrecDesc*, GKVecs<double>, GKState*, GKWork&, hipStream_t);
template void gk_iteration<float>(const OpDesc&, const PrecDesc*, GKVecs<float>, GKState*, GKWork&, hipStream_t);
template void gk_phase_init<double>(const OpDesc&, const OpDesc&, const PrecDesc*, const double*, const double*,
                                    double, const double*, GKVecs<double>, GKState*, GKWork&, hipStream_t);
template void gk_phase_init<float>(const OpDesc&, const OpDesc&, const PrecDesc*, const double*, const double*,
                                   double, const double*, GKVecs<float>, GKState*, GKWork&, hipStream_t);
template void gk_phase_finish<double>(const OpDesc&, const PrecDesc*, GKVecs<double>, double*, GKState*,
                                      hipStream_t);
template void gk_phase_finish<float>(const OpDesc&, const PrecDesc*, GKVecs<float>, double*, GKState*,
                                     hipStream_t);

// ||A_mu^T r||^2 -> slot 0 h2 for r = [b - A x; bot_scale b_bot - delta x]:
// the plain phase start followed by its initial scalar step.
void gk_normal_residual(const OpDesc& A, const double* b, const double* b_bot, double bot_scale, const double* x,
                        GKVecs<double> vec, GKState* st, GKWork& wk, hipStream_t s) {
  launch_resid<double>(A, b, b_bot, bot_scale, x, vec.u_top, vec.u_bot, st, wk, s);
  launch_bwd<double, true>(A, vec.u_top, vec.u_bot, vec.v, vec.g, st, wk, true, s);
  hipLaunchKernelGGL(k_consume, dim3(1), dim3(kBlock), 0, s, st, (const double*)wk.alpha_part, (int)wk.alpha_count,
                     0);
}

// g = A_mu^T [b - A x; bot_scale b_bot - delta x] in FP64 (state: beta = 1);
// r_top, r_bot receive the residual.
void gk_normal_vector(const OpDesc& A, const double* b, const double* b_bot, double bot_scale, const double* x,
                      double* r_top, double* r_bot, double* g, GKState* st, GKWork& wk, hipStream_t s) {
  launch_resid<double>(A, b, b_bot, bot_scale, x, r_top, r_bot, st, wk, s);
  launch_bwd<double, false>(A, r_top, r_bot, nullptr, g, st, wk, false, s);
}

// Both state slots <- h (by value through the kernel arguments, so the host
// copy may change as soon as the launch returns).
__global__ void k_set_state(GKState* st, GKState h) {
  if (threadIdx.x == 0) {
    st[0] = h;
    st[1] = h;
  }
}

void set_state(GKState* st, const GKState& h, hipStream_t s) {
  hipLaunchKernelGGL(k_set_state, dim3(1), dim3(64), 0, s, st, h);
}

// ||A^T b||^2 -> slot 0 h2 (state: beta = 1, delta = 0, init = 1).
void op_atb_norm2(const OpDesc& A, const double* b, double* tmp_n, GKState* st, GKWork& wk, hipStream_t s) {
  launch_bwd<double, false>(A, b, nullptr, nullptr, tmp_n, st, wk, false, s);
  hipLaunchKernelGGL(k_consume, dim3(1), dim3(kBlock), 0, s, st, (const double*)wk.alpha_part, (int)wk.alpha_count,
                     0);
}

// ||[b; bot_scale b_bot]|| -> slot 0 beta (state: init = 1; the bottom part
// counts only when the state's delta > 0; b or b_bot may be null = 0).
void op_norm(const OpDesc& A, const double* b, const double* b_bot, double bot_scale, double* tmp_m, double* tmp_n,
             GKState* st, GKWork& wk, hipStream_t s) {
  launch_resid<double>(A, b, b_bot, bot_scale, nullptr, tmp_m, tmp_n, st, wk, s);
  hipLaunchKernelGGL(k_consume, dim3(1), dim3(kBlock), 0, s, st, (const double*)wk.beta_part, (int)wk.beta_count, 1);
}

// y = A x - y_prev (trans = 0: the LSQR forward kernel with alpha = beta = 1,
// delta = 0) or y = A^T x (trans = 1); the slots hold that state.  With
// events e0/e1 the product's own start and end are recorded.
void op_matvec(const OpDesc& A, int trans, const double* x, double* y, GKState* st, GKWork& wk, hipStream_t s,
               hipEvent_t e0, hipEvent_t e1) {
  if (!trans) {
    GKVecs<double> vec{y, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    launch_fwd<double, kFwdMatvec>(A, x, vec, st, wk, s, e0, e1);
  } else {
    launch_bwd<double, false>(A, x, nullptr, nullptr, y, st, wk, false, s, e0, e1);
  }
}

}  // namespace aplicur
