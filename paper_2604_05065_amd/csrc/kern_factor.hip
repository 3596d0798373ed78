// Kernels of the CUR part of APLICUR (Alg. 3 Parts 1-3): LU-with-partial-
// pivoting pivot selection (Alg. 7), gathers of rows/columns of A, small
// dense factorisations (Cholesky, Gauss-Jordan inverse) and the one-sided
// block Jacobi SVD of the l x l core M (Alg. 2).  All FP64.
#include "factor.h"

namespace aplicur {

// ============================================================== LUPP pivots
// Partial-pivoting elimination on a column-major r x c matrix X, keeping the
// LAPACK row order for ties: pos[i] is the current position of original row
// i and row_at[p] its inverse (rows are not moved; only this bookkeeping
// is).  The pivot of column q is the remaining row with the largest
// |X(i,q)|, the smallest position winning ties (as idamax does).  One launch
// per column: every workgroup reduces the previous launch's per-workgroup
// argmax candidates itself (fixed order, no fences), applies the row swap of
// step q to double-buffered copies of pos/row_at, eliminates column q and
// proposes the pivot candidates of column q + 1.
struct LuppState {
  int keff;  // pivots found so far
  int stop;  // set when done or when a pivot column is zero (exhausted)
};

__device__ __forceinline__ bool better(double va, int pa, double vb, int pb) {
  return va > vb || (va == vb && pa < pb);
}

// The workgroup's best (value, position, row) by `better`: a butterfly over
// each wave's lanes, then the waves' results in order.  `better` is a total
// order on distinct positions, so the result does not depend on the tree.
__device__ void block_argmax(double& v, int& p, int& idx) {
  constexpr int NW = kBlock / kWave;
  __shared__ double sv[NW];
  __shared__ int sp[NW], si[NW];
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    const double ov = __shfl_xor(v, off, kWave);
    const int op = __shfl_xor(p, off, kWave);
    const int oi = __shfl_xor(idx, off, kWave);
    if (better(ov, op, v, p)) {
      v = ov;
      p = op;
      idx = oi;
    }
  }
  if (threadIdx.x % kWave == 0) {
    sv[threadIdx.x / kWave] = v;
    sp[threadIdx.x / kWave] = p;
    si[threadIdx.x / kWave] = idx;
  }
  __syncthreads();
  v = sv[0];
  p = sp[0];
  idx = si[0];
#pragma unroll
  for (int w = 1; w < NW; ++w)
    if (better(sv[w], sp[w], v, p)) {
      v = sv[w];
      p = sp[w];
      idx = si[w];
    }
  __syncthreads();
}

// Every workgroup: the global best of the previous launch's candidates.
__device__ void argmax_all(const double* pv, const int* pp, const int* pi, int count, double& v, int& idx) {
  double bv = -1.0;
  int bp = INT_MAX, bi = -1;
  for (int t = threadIdx.x; t < count; t += kBlock)
    if (better(pv[t], pp[t], bv, bp)) {
      bv = pv[t];
      bp = pp[t];
      bi = pi[t];
    }
  block_argmax(bv, bp, bi);
  v = bv;
  idx = bi;
}

__global__ void __launch_bounds__(kBlock) k_lupp_init(const double* X, int r, int k, int* pos, int* row_at,
                                                      LuppState* ls, double* pv, int* pp, int* pi) {
  double v = -1.0;
  int p = INT_MAX, idx = -1;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < r; i += gridDim.x * kBlock) {
    pos[i] = i;
    row_at[i] = i;
    const double a = fabs(X[i]);
    if (better(a, i, v, p)) {
      v = a;
      p = i;
      idx = i;
    }
  }
  block_argmax(v, p, idx);
  if (threadIdx.x == 0) {
    pv[blockIdx.x] = v;
    pp[blockIdx.x] = p;
    pi[blockIdx.x] = idx;
    if (blockIdx.x == 0) {
      ls->keff = 0;
      ls->stop = (k <= 0);
    }
  }
}

constexpr int kLuppUnroll = 16;  // columns of a row updated per batch of loads

// One pivot step: the global best of the previous candidates is the pivot
// (original row p) of position q; positions are updated as if the rows were
// swapped (LAPACK order); the multipliers of the remaining rows are stored in
// column q and columns q + 1 .. cend - 1 are eliminated; candidates for column
// q + 1 are produced when q + 1 < cend (otherwise k_lupp_cand makes them after
// the trailing update of a blocked factorisation).
__global__ void __launch_bounds__(kBlock)
    k_lupp_step(double* X, int r, int c, int cend, long long ld, int q, int k, const int* pos_cur,
                const int* row_cur, int* pos_nxt, int* row_nxt, int* piv, LuppState* ls, const double* pv_in,
                const int* pp_in, const int* pi_in, double* pv_out, int* pp_out, int* pi_out) {
  if (ls->stop) return;
  double vmax;
  int p;
  argmax_all(pv_in, pp_in, pi_in, gridDim.x, vmax, p);
  if (!(vmax > 0.0) || p < 0) {  // zero (or NaN) pivot column: residual exhausted
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      ls->keff = q;
      ls->stop = 1;
    }
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    piv[q] = p;
    ls->keff = q + 1;
    if (q + 1 >= k || q + 1 >= c) ls->stop = 1;
  }
  if (q + 1 >= k || q + 1 >= c) return;  // last pivot found: no elimination needed
  const int o = row_cur[q];               // row currently at position q
  const int pp = pos_cur[p];              // current position of the pivot row
  const double piv_val = X[p + q * ld];
  double v = -1.0;
  int bp = INT_MAX, idx = -1;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < r; i += gridDim.x * kBlock) {
    const int pi_old = pos_cur[i];
    const int pn = (i == p) ? q : ((i == o) ? pp : pi_old);
    pos_nxt[i] = pn;
    row_nxt[i] = (i == q) ? p : ((i == pp) ? o : row_cur[i]);
    if (pn <= q) continue;  // pivot rows (positions 0..q) are not updated
    const double l = X[i + q * ld] / piv_val;
    X[i + q * ld] = l;
    // the row's entries and the pivot row's, kLuppUnroll columns at a time,
    // all loaded before any is updated (independent loads in flight)
    double first = 0.0;
    for (int j0 = q + 1; j0 < cend; j0 += kLuppUnroll) {
      double xv[kLuppUnroll], pr[kLuppUnroll];
#pragma unroll
      for (int u = 0; u < kLuppUnroll; ++u) {
        const int j = j0 + u;
        xv[u] = j < cend ? X[i + j * ld] : 0.0;
        pr[u] = j < cend ? X[p + j * ld] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kLuppUnroll; ++u) {
        const int j = j0 + u;
        if (j < cend) {
          const double nv = xv[u] - l * pr[u];
          X[i + j * ld] = nv;
          if (j == q + 1) first = nv;
        }
      }
    }
    if (q + 1 < cend) {
      const double a = fabs(first);
      if (better(a, pn, v, bp)) {
        v = a;
        bp = pn;
        idx = i;
      }
    }
  }
  if (q + 1 >= cend) return;  // uniform
  block_argmax(v, bp, idx);
  if (threadIdx.x == 0) {
    pv_out[blockIdx.x] = v;
    pp_out[blockIdx.x] = bp;
    pi_out[blockIdx.x] = idx;
  }
}

// Candidates for the pivot of column col among the rows at positions >= col.
__global__ void __launch_bounds__(kBlock) k_lupp_cand(const double* X, int r, long long ld, int col, const int* pos,
                                                      const LuppState* ls, double* pv, int* pp, int* pi) {
  if (ls->stop) return;
  double v = -1.0;
  int bp = INT_MAX, idx = -1;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < r; i += gridDim.x * kBlock) {
    const int pn = pos[i];
    if (pn < col) continue;
    const double a = fabs(X[i + col * ld]);
    if (better(a, pn, v, bp)) {
      v = a;
      bp = pn;
      idx = i;
    }
  }
  block_argmax(v, bp, idx);
  if (threadIdx.x == 0) {
    pv[blockIdx.x] = v;
    pp[blockIdx.x] = bp;
    pi[blockIdx.x] = idx;
  }
}

// G (nb x w, column-major) = X(piv[q0 .. q0 + nb), q0 .. q0 + w) (row indices clamped into range).
__global__ void k_lupp_gather(const double* X, int r, long long ld, const int* piv, int q0, int nb, int w,
                              double* G) {
  for (int e = blockIdx.x * kBlock + threadIdx.x; e < nb * w; e += gridDim.x * kBlock) {
    const int qq = e % nb, j = e / nb;
    int p = piv[q0 + qq];
    p = (p < 0 || p >= r) ? 0 : p;
    G[e] = X[p + (long long)(q0 + j) * ld];
  }
}

static int lupp_grid(int r) { return std::min((r + kBlock - 1) / kBlock, 1024); }

void lupp_begin(double* X, int r, int k, FactorWork& fw, hipStream_t s) {
  APL_REQUIRE(r <= fw.lupp_rows, "lupp: workspace rows too small");
  LuppState* ls = (LuppState*)fw.lupp_state;
  hipLaunchKernelGGL(k_lupp_init, dim3(lupp_grid(r)), dim3(kBlock), 0, s, X, r, k, fw.pos, fw.row_at, ls, fw.pv,
                     fw.pp, fw.pi);
}

// Buffers of step q: positions / rows and candidates are double-buffered by q % 2.
void lupp_step(double* X, int r, int c, int cend, long long ld, int q, int k, int* piv, FactorWork& fw,
               hipStream_t s) {
  const int a = q & 1, b = a ^ 1;
  int* pos[2] = {fw.pos, fw.pos + r};
  int* row[2] = {fw.row_at, fw.row_at + r};
  double* pv[2] = {fw.pv, fw.pv + 1024};
  int* pp[2] = {fw.pp, fw.pp + 1024};
  int* pi[2] = {fw.pi, fw.pi + 1024};
  hipLaunchKernelGGL(k_lupp_step, dim3(lupp_grid(r)), dim3(kBlock), 0, s, X, r, c, cend, ld, q, k, pos[a], row[a],
                     pos[b], row[b], piv, (LuppState*)fw.lupp_state, pv[a], pp[a], pi[a], pv[b], pp[b], pi[b]);
}

void lupp_cand(const double* X, int r, long long ld, int col, FactorWork& fw, hipStream_t s) {
  const int a = col & 1;
  int* pos = a ? fw.pos + r : fw.pos;
  double* pv = fw.pv + (a ? 1024 : 0);
  int* pp = fw.pp + (a ? 1024 : 0);
  int* pi = fw.pi + (a ? 1024 : 0);
  hipLaunchKernelGGL(k_lupp_cand, dim3(lupp_grid(r)), dim3(kBlock), 0, s, X, r, ld, col, (const int*)pos,
                     (const LuppState*)fw.lupp_state, pv, pp, pi);
}

void lupp_gather(const double* X, int r, long long ld, const int* piv, int q0, int nb, int w, double* G,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_lupp_gather, dim3(std::min<unsigned>(ceil_div((long long)nb * w, kBlock), 256)), dim3(kBlock),
                     0, s, X, r, ld, piv, q0, nb, w, G);
}

void lupp_pivots(double* X, int r, int c, long long ld, int k, int* piv, FactorWork& fw, hipStream_t s) {
  lupp_begin(X, r, k, fw, s);
  for (int q = 0; q < k; ++q) lupp_step(X, r, c, c, ld, q, k, piv, fw, s);
}

int lupp_read_keff(FactorWork& fw, hipStream_t s) {
  LuppState h;
  APL_HIP(hipMemcpyAsync(&h, fw.lupp_state, sizeof(h), hipMemcpyDeviceToHost, s));
  APL_HIP(hipStreamSynchronize(s));
  return h.keff;
}

// ============================================================== gathers
// out(i, t) = A(i, J[t]) for dense row-major A (column-major out, ld_out).
template <class T>
__global__ void k_gather_cols_dense(const T* A, long long m, long long ld, const int* J, int k,
                                    double* out, long long ld_out) {
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  const int t = blockIdx.y;
  if (i < m && t < k) out[i + t * ld_out] = (double)A[i * ld + J[t]];
}

// out(:, t) = A(:, J[t]) for CSR A through its transpose (rows of A^T).
template <class T>
__global__ void k_gather_cols_csr(const int* tp, const int* ti, const T* tv, const int* J, int k,
                                  double* out, long long ld_out) {
  const int t = blockIdx.x;
  if (t >= k) return;
  const int j = J[t];
  for (int e = tp[j] + threadIdx.x; e < tp[j + 1]; e += kBlock) out[ti[e] + t * ld_out] = (double)tv[e];
}

// out(j, t) = A(I[t], j): rows of A as columns of a column-major n x k block.
template <class T>
__global__ void k_gather_rows_dense(const T* A, long long n, long long ld, const int* I, int k,
                                    double* out, long long ld_out) {
  const long long j = (long long)blockIdx.x * kBlock + threadIdx.x;
  const int t = blockIdx.y;
  if (j < n && t < k) out[j + t * ld_out] = (double)A[(long long)I[t] * ld + j];
}

template <class T>
__global__ void k_gather_rows_csr(const int* rp, const int* ci, const T* val, const int* I, int k,
                                  double* out, long long ld_out) {
  const int t = blockIdx.x;
  if (t >= k) return;
  const int i = I[t];
  for (int e = rp[i] + threadIdx.x; e < rp[i + 1]; e += kBlock) out[ci[e] + t * ld_out] = (double)val[e];
}

// out(a, t) = X(rows[a], t) for a < nr: gather rows of a column-major matrix.
__global__ void k_gather_sub_rows(const double* X, long long ldx, const int* rows, int nr, int ncols,
                                  double* out, long long ldo) {
  const int a = blockIdx.x * kBlock + threadIdx.x;
  const int t = blockIdx.y;
  if (a < nr && t < ncols) out[a + t * ldo] = X[rows[a] + t * ldx];
}

// X(rows[a], t) = 0 for every column t < ncols.
__global__ void k_zero_rows(double* X, long long ldx, const int* rows, int nr, int ncols) {
  const int a = blockIdx.x * kBlock + threadIdx.x;
  const int t = blockIdx.y;
  if (a < nr && t < ncols) X[rows[a] + t * ldx] = 0.0;
}

__global__ void k_fill(double* X, long long n, double v) {
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
    X[i] = v;
}

// Y(h, j) row-major s x n  ->  column-major s x k block of the columns J.
__global__ void k_gather_y_cols(const double* Y, long long n, int s, const int* J, int k, double* out,
                                long long ldo) {
  const int h = blockIdx.x * kBlock + threadIdx.x;
  const int t = blockIdx.y;
  if (h < s && t < k) out[h + t * ldo] = Y[(long long)h * n + J[t]];
}

void gather_cols(const AMat& A, const int* J, int k, double* out, long long ld_out, hipStream_t s) {
  if (k <= 0) return;
  if (A.csr) {
    fill(out, ld_out * (long long)(k - 1) + A.m, 0.0, s);
    if (A.f64)
      hipLaunchKernelGGL(k_gather_cols_csr<double>, dim3(k), dim3(kBlock), 0, s, A.t_ptr, A.t_idx,
                         (const double*)A.t_val, J, k, out, ld_out);
    else
      hipLaunchKernelGGL(k_gather_cols_csr<float>, dim3(k), dim3(kBlock), 0, s, A.t_ptr, A.t_idx,
                         (const float*)A.t_val, J, k, out, ld_out);
  } else {
    dim3 g(ceil_div(A.m, kBlock), k);
    if (A.f64)
      hipLaunchKernelGGL(k_gather_cols_dense<double>, g, dim3(kBlock), 0, s, (const double*)A.val, A.m, A.ld,
                         J, k, out, ld_out);
    else
      hipLaunchKernelGGL(k_gather_cols_dense<float>, g, dim3(kBlock), 0, s, (const float*)A.val, A.m, A.ld,
                         J, k, out, ld_out);
  }
}

void gather_rows(const AMat& A, const int* I, int k, double* out, long long ld_out, hipStream_t s) {
  if (k <= 0) return;
  if (A.csr) {
    fill(out, ld_out * (long long)(k - 1) + A.n, 0.0, s);
    if (A.f64)
      hipLaunchKernelGGL(k_gather_rows_csr<double>, dim3(k), dim3(kBlock), 0, s, A.row_ptr, A.col_idx,
                         (const double*)A.val, I, k, out, ld_out);
    else
      hipLaunchKernelGGL(k_gather_rows_csr<float>, dim3(k), dim3(kBlock), 0, s, A.row_ptr, A.col_idx,
                         (const float*)A.val, I, k, out, ld_out);
  } else {
    dim3 g(ceil_div(A.n, kBlock), k);
    if (A.f64)
      hipLaunchKernelGGL(k_gather_rows_dense<double>, g, dim3(kBlock), 0, s, (const double*)A.val, A.n, A.ld,
                         I, k, out, ld_out);
    else
      hipLaunchKernelGGL(k_gather_rows_dense<float>, g, dim3(kBlock), 0, s, (const float*)A.val, A.n, A.ld,
                         I, k, out, ld_out);
  }
}

void gather_sub_rows(const double* X, long long ldx, const int* rows, int nr, int ncols, double* out,
                     long long ldo, hipStream_t s) {
  if (nr <= 0 || ncols <= 0) return;
  hipLaunchKernelGGL(k_gather_sub_rows, dim3(ceil_div(nr, kBlock), ncols), dim3(kBlock), 0, s, X, ldx, rows,
                     nr, ncols, out, ldo);
}

void zero_rows(double* X, long long ldx, const int* rows, int nr, int ncols, hipStream_t s) {
  if (nr <= 0 || ncols <= 0) return;
  hipLaunchKernelGGL(k_zero_rows, dim3(ceil_div(nr, kBlock), ncols), dim3(kBlock), 0, s, X, ldx, rows, nr,
                     ncols);
}

// Adds one to every 32-bit word of buf (bytes a multiple of 16): a read and a
// write of the whole buffer, which evicts other data from the caches.
__global__ void k_touch(uint4* buf, long long n16) {
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n16; i += (long long)gridDim.x * kBlock) {
    uint4 v = buf[i];
    v.x += 1u;
    v.y += 1u;
    v.z += 1u;
    v.w += 1u;
    buf[i] = v;
  }
}

void touch_buffer(void* buf, long long bytes, hipStream_t s) {
  const long long n16 = bytes / 16;
  hipLaunchKernelGGL(k_touch, dim3((unsigned)std::min<long long>(ceil_div(n16, kBlock), 8192)), dim3(kBlock), 0, s,
                     (uint4*)buf, n16);
}

void fill(double* X, long long n, double v, hipStream_t s) {
  if (n <= 0) return;
  unsigned g = ceil_div(n, kBlock);
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_fill, dim3(g), dim3(kBlock), 0, s, X, n, v);
}

void gather_y_cols(const double* Y, long long n, int s_rows, const int* J, int k, double* out, long long ldo,
                   hipStream_t s) {
  if (k <= 0) return;
  hipLaunchKernelGGL(k_gather_y_cols, dim3(ceil_div(s_rows, kBlock), k), dim3(kBlock), 0, s, Y, n, s_rows, J,
                     k, out, ldo);
}

// ============================================================== blocked small factorisations
// The diagonal-block and panel kernels of the blocked Cholesky and LU below
// (their trailing updates are library TRSM / SYRK / GEMM calls): one
// workgroup of kFT threads with the block in LDS.
constexpr int kFT = 1024;

// Upper Cholesky of the nb x nb diagonal block at G (column-major, ld): U^T U
// = G in place (upper triangle; the strict lower triangle is left alone).
// status[0] = 1 + (j0 + j) if pivot j is not positive; nothing is done when
// status[0] is already set.  The block stays in registers: lane i holds row
// i of the columns w, w + 16, w + 32, w + 48 of wave w.  Step j reads row j
// of the current matrix from LDS (published by the lanes that own it at the
// end of step j - 1, double-buffered), forms r = sqrt(g_jj) and the scaled
// row u = g_j. / r (lane x divides entry x; the others come by readlane),
// makes row j that row of U (diagonal r) and updates g_xy -= u_x u_y for j <
// x <= y; one barrier per step.
constexpr int kPW = kFT / kWave;        // waves of the register-resident block kernels
constexpr int kPCols = kFNB / kPW;      // columns per wave
static_assert(kFNB == kWave && kFNB % kPW == 0, "register-resident blocks: kFNB rows, one per lane");
__global__ void __launch_bounds__(kFT) k_potrf_diag(double* G, long long ld, int nb, int j0, int* status) {
  __shared__ double row[2][kFNB];
  __shared__ int bad;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  if (threadIdx.x == 0) bad = status[0];
  double x[kPCols];
#pragma unroll
  for (int b = 0; b < kPCols; ++b) {
    const int y = wave + kPW * b;
    x[b] = (lane <= y && y < nb) ? G[lane + (long long)y * ld] : 0.0;
    if (lane == 0) row[0][y] = x[b];
  }
  __syncthreads();
  if (bad) return;  // uniform
  for (int j = 0; j < nb; ++j) {
    const int par = j & 1;
    const double d = row[par][j];
    if (!(d > 0.0)) {
      if (threadIdx.x == 0) status[0] = 1 + j0 + j;
      return;  // uniform: every thread read the same d
    }
    const double r = sqrt(d);
    const double u = row[par][lane] / r;  // u_x for x = lane; u_y from lane y
#pragma unroll
    for (int b = 0; b < kPCols; ++b) {
      const int y = wave + kPW * b;
      if (y >= nb || y < j) continue;
      const double uy = lane_bcast(u, y);
      if (lane == j) {
        x[b] = y == j ? r : uy;
      } else if (lane > j && lane <= y) {
        x[b] -= u * uy;
      }
      if (lane == j + 1 && y >= j + 1) row[par ^ 1][y] = x[b];
    }
    __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < kPCols; ++b) {
    const int y = wave + kPW * b;
    if (lane <= y && y < nb) G[lane + (long long)y * ld] = x[b];
  }
}

void potrf_diag(double* G, long long ld, int nb, int j0, int* status, hipStream_t s) {
  APL_REQUIRE(nb >= 1 && nb <= kFNB, "potrf_diag: block too large");
  hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(kFT), 0, s, G, ld, nb, j0, status);
}

// LU with partial pivoting (first largest magnitude) of the panel
// A[j0:k, j0:j0+w] (column-major, ld; k - j0 <= kFMaxRows, w <= kFNB):
// piv[j0 + c] = the row swapped with row j0 + c; L below the diagonal (unit),
// U on and above.  status[0] = 1 if a pivot is zero (the elimination of that
// column is skipped).  The panel stays in registers: lane i holds rows i,
// i + 64, ... of the columns w, w + 16, w + 32, w + 48 of wave w.  Column c
// belongs to one wave, which finds the pivot (a wave reduction), swaps the
// two rows in its columns, scales the multipliers and publishes them, the
// pivot row and the pivot through LDS (double-buffered); after the step's
// one barrier every other wave swaps the two rows in its columns (lane reads
// and writes, the rows being uniform) and updates its columns right of c.
constexpr int kLuRows = (kFMaxRows + kWave - 1) / kWave;  // rows per lane
static_assert(kFNB <= kWave, "k_lu_panel: the panel's pivot rows (c < w <= kFNB) sit in the first row slot");
__global__ void __launch_bounds__(kFT) k_lu_panel(double* A, long long ld, int k, int j0, int w, int* piv,
                                                  int* status) {
  __shared__ double mult[2][kLuRows * kWave];
  __shared__ double s_d[2];
  __shared__ int s_pr[2];
  __shared__ double prow[kPW][kPCols];  // per wave: the pivot row's entries before the swap
  const int R = k - j0;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  double x[kPCols][kLuRows];
#pragma unroll
  for (int b = 0; b < kPCols; ++b) {
    const int j = wave + kPW * b;
#pragma unroll
    for (int a = 0; a < kLuRows; ++a) {
      const int r = lane + kWave * a;
      x[b][a] = (r < R && j < w) ? A[(j0 + r) + (long long)(j0 + j) * ld] : 0.0;
    }
  }
  // Rows c (slot 0 of lane c, as c < kWave) and pr exchanged in this wave's
  // columns: row pr's entries pass through the wave's LDS row (written by
  // its owner lane, read back by every lane: in order within the wave).
  auto swap_rows = [&](int c, int pr) {
    if (pr == c) return;
#pragma unroll
    for (int a = 0; a < kLuRows; ++a)
      if (lane + kWave * a == pr) {
#pragma unroll
        for (int b = 0; b < kPCols; ++b) prow[wave][b] = x[b][a];
      }
    double vc[kPCols];
#pragma unroll
    for (int b = 0; b < kPCols; ++b) vc[b] = lane_bcast(x[b][0], c);
#pragma unroll
    for (int b = 0; b < kPCols; ++b) {
      const double vp = prow[wave][b];
      if (lane == c) x[b][0] = vp;
#pragma unroll
      for (int a = 0; a < kLuRows; ++a)
        if (lane + kWave * a == pr) x[b][a] = vc[b];
    }
  };
#pragma unroll
  for (int bc = 0; bc < kPCols; ++bc) {
    for (int wc = 0; wc < kPW; ++wc) {
      const int c = kPW * bc + wc;
      if (c >= w) break;  // uniform
      const int par = c & 1;
      if (wave == wc) {
        // argmax |A(r, c)| over r in [c, R), smallest index on ties
        double v = -1.0;
        int idx = INT_MAX;
#pragma unroll
        for (int a = 0; a < kLuRows; ++a) {
          const int r = lane + kWave * a;
          if (r >= c && r < R) {
            const double t = fabs(x[bc][a]);
            if (t > v) {
              v = t;
              idx = r;
            }
          }
        }
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) {
          const double ov = __shfl_xor(v, off, kWave);
          const int oi = __shfl_xor(idx, off, kWave);
          if (ov > v || (ov == v && oi < idx)) {
            v = ov;
            idx = oi;
          }
        }
        if (idx == INT_MAX) idx = c;  // no comparable entry (NaN): no swap, and status flags it
        const int pr = __builtin_amdgcn_readfirstlane(idx);
        if (lane == 0) {
          piv[j0 + c] = j0 + pr;
          if (!(v > 0.0)) status[0] = 1;
        }
        swap_rows(c, pr);
        const double d = lane_bcast(x[bc][0], c);
        if (d != 0.0) {
          const double inv = 1.0 / d;
#pragma unroll
          for (int a = 0; a < kLuRows; ++a) {
            const int r = lane + kWave * a;
            if (r > c && r < R) x[bc][a] *= inv;
          }
        }
#pragma unroll
        for (int a = 0; a < kLuRows; ++a) mult[par][lane + kWave * a] = x[bc][a];
        if (lane == 0) {
          s_pr[par] = pr;
          s_d[par] = d;
        }
      }
      __syncthreads();
      const int pr = __builtin_amdgcn_readfirstlane(s_pr[par]);
      const double d = s_d[par];
      if (wave != wc) swap_rows(c, pr);
      if (d != 0.0) {
#pragma unroll
        for (int b = 0; b < kPCols; ++b) {
          const int j = wave + kPW * b;
          if (j <= c || j >= w) continue;
          const double pc = lane_bcast(x[b][0], c);
#pragma unroll
          for (int a = 0; a < kLuRows; ++a) {
            const int r = lane + kWave * a;
            if (r > c && r < R) x[b][a] -= mult[par][r] * pc;
          }
        }
      }
    }
  }
#pragma unroll
  for (int b = 0; b < kPCols; ++b) {
    const int j = wave + kPW * b;
#pragma unroll
    for (int a = 0; a < kLuRows; ++a) {
      const int r = lane + kWave * a;
      if (r < R && j < w) A[(j0 + r) + (long long)(j0 + j) * ld] = x[b][a];
    }
  }
}

// Row swaps piv[j0 .. j0 + w) (in order) on the columns outside [c0, c1) of
// the k x ncols matrix A (column-major, ld): one thread per column.
__global__ void k_laswp(double* A, long long ld, int ncols, int c0, int c1, const int* piv, int j0, int w) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= ncols || (j >= c0 && j < c1)) return;
  double* col = A + (long long)j * ld;
  for (int c = 0; c < w; ++c) {
    const int r = j0 + c, q = piv[j0 + c];
    if (q != r) {
      const double t = col[r];
      col[r] = col[q];
      col[q] = t;
    }
  }
}

void lu_panel(double* A, long long ld, int k, int j0, int w, int* piv, int* status, hipStream_t s) {
  APL_REQUIRE(k - j0 <= kFMaxRows && w >= 1 && w <= kFNB && w <= k - j0, "lu_panel: panel too large");
  hipLaunchKernelGGL(k_lu_panel, dim3(1), dim3(kFT), 0, s, A, ld, k, j0, w, piv, status);
}

void laswp(double* A, long long ld, int ncols, int c0, int c1, const int* piv, int j0, int w, hipStream_t s) {
  hipLaunchKernelGGL(k_laswp, dim3(ceil_div(ncols, kBlock)), dim3(kBlock), 0, s, A, ld, ncols, c0, c1, piv, j0, w);
}

__global__ void k_zero_lower(double* G, long long ld, int k) {
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < (long long)k * k;
       e += (long long)gridDim.x * kBlock) {
    const int i = (int)(e % k), j = (int)(e / k);
    if (i > j) G[i + (long long)j * ld] = 0.0;
  }
}

void zero_lower(double* G, long long ld, int k, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_lower, dim3(std::min<unsigned>(ceil_div((long long)k * k, kBlock), 256)), dim3(kBlock), 0,
                     s, G, ld, k);
}

typedef double f64x4_t __attribute__((ext_vector_type(4)));

// ============================================================== block one-sided Jacobi SVD
// X (rows x npad, column-major) is orthogonalised column-block-pair by
// column-block-pair (Hestenes' method, block form): for the pair of blocks
// (a, b), 2 kJW columns, the Gram matrix is formed, one cyclic Jacobi sweep
// diagonalises it approximately, and the rotation Q is applied to those
// columns of X and of V.  Round-robin (circle) pairing covers every block pair
// once per sweep; the pairs of a round touch disjoint columns.  One round is
// three launches:
//   k_jac_gram   row chunks x pairs: partial Gram matrices of the pair's
//                columns over a chunk of rows (FP64 16x16x4 MFMA);
//   k_jac_rot    one workgroup per pair: the partials summed in chunk order,
//                the off-diagonal measure, the inner sweep in LDS, Q stored;
//   k_jac_apply  row chunks x pairs x {X, V}: rows times Q on the MFMA, in
//                place (a wave reads its rows' pair columns before writing).
// Off-diagonal entries are measured on the damped Gram matrix X^T X + d2 I
// (d2 = delta^2: the columns of the damped core [X; delta V], whose right
// singular vectors are X's): e_pq = |g_pq| / sqrt((g_pp + d2)(g_qq + d2)).
// sq_part[round * npairs + pair] receives the sum of e_pq^2 over the entries
// between the pair's two blocks, so that a sweep's partials cover each such
// entry once; they are summed afterwards in a fixed order.  A pair whose
// largest e_pq is at most `skip` leaves X and V as they are.
constexpr int kJW = 16;       // columns per block
constexpr int kJP = 2 * kJW;  // columns per pair
constexpr int kJT = 256;      // threads per workgroup (4 waves)
constexpr int kJMaxChunks = 16;
constexpr int kJAJ = 1;       // 16-row tiles per wave in k_jac_apply
constexpr int kJARows = (kJT / kWave) * 16 * kJAJ;  // rows per workgroup of k_jac_apply
static_assert(kJP % 16 == 0 && (kJP / 16) * (kJP / 16) <= 4, "pair Gram: at most one 16x16 tile per wave");

__device__ __forceinline__ void pair_of(int round, int nblk, int slot, int& a, int& b) {
  // circle method: block nblk-1 fixed, the others rotate
  if (slot == 0) {
    a = nblk - 1;
    b = round % (nblk - 1);
  } else {
    a = (round + slot) % (nblk - 1);
    b = (round - slot + (nblk - 1)) % (nblk - 1);
  }
  if (a > b) {
    int t = a;
    a = b;
    b = t;
  }
}

// column of X of the pair's column c (block a's kJW columns, then block b's)
__device__ __forceinline__ int pair_col(int a, int b, int c) { return c < kJW ? a * kJW + c : b * kJW + (c - kJW); }

// Partial Gram of the pair's columns over rows [chunk * rpc, ...): each wave
// forms all (kJP/16)^2 16x16 tiles over the 16-row steps wave, wave + 4, ...
// (lane (i, q) loads column i of each 16-column slab at rows 4q .. 4q + 3 of
// the step, which serve as the A operand of the slab's tile rows and the B
// operand of its tile columns); the waves' partials are summed in wave
// order.  gpart[(pair * nchunk + chunk) * kJP^2 + i kJP + j].
__global__ void __launch_bounds__(kJT) k_jac_gram(const double* __restrict__ X, long long ldx, int rows, int nblk,
                                                   int round, int rpc, int nchunk, double* __restrict__ gpart) {
  constexpr int NT = kJP / 16, NW = kJT / kWave;
  __shared__ double red[NW][kJP][kJP + 1];
  const int chunk = blockIdx.x, pair = blockIdx.y;
  int a, b;
  pair_of(round, nblk, pair, a, b);
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave, li = lane % 16, lq = lane / 16;
  const double* xs[NT];
#pragma unroll
  for (int s = 0; s < NT; ++s) xs[s] = X + (long long)pair_col(a, b, s * 16 + li) * ldx;
  const int r_begin = chunk * rpc, r_end = min(rows, r_begin + rpc);
  f64x4_t acc[NT][NT];
#pragma unroll
  for (int ti = 0; ti < NT; ++ti)
#pragma unroll
    for (int tj = 0; tj < NT; ++tj) acc[ti][tj] = (f64x4_t){0.0, 0.0, 0.0, 0.0};
  constexpr int kU = 2;  // 16-row steps in flight per wave
  for (int r0 = r_begin + wave * 16; r0 < r_end; r0 += NW * 16 * kU) {
    double v[kU][NT][4];
#pragma unroll
    for (int u = 0; u < kU; ++u)
#pragma unroll
      for (int s = 0; s < NT; ++s)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = r0 + u * NW * 16 + 4 * lq + e;
          v[u][s][e] = r < r_end ? xs[s][r] : 0.0;
        }
#pragma unroll
    for (int u = 0; u < kU; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int ti = 0; ti < NT; ++ti)
#pragma unroll
          for (int tj = 0; tj < NT; ++tj)
            acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[u][ti][e], v[u][tj][e], acc[ti][tj], 0, 0, 0);
  }
  // register r of lane (i, q) holds G[ti 16 + q + 4r][tj 16 + i]
#pragma unroll
  for (int ti = 0; ti < NT; ++ti)
#pragma unroll
    for (int tj = 0; tj < NT; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[wave][ti * 16 + lq + 4 * r][tj * 16 + li] = acc[ti][tj][r];
  __syncthreads();
  double* out = gpart + ((long long)pair * nchunk + chunk) * (kJP * kJP);
  for (int e = threadIdx.x; e < kJP * kJP; e += kJT) {
    const int i = e / kJP, j = e % kJP;
    double g = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) g += red[w][i][j];
    out[e] = g;
  }
}

// Partner of index i in step r of a cyclic sweep over kJP indices (circle
// method: index kJP - 1 fixed, the others rotate).
__device__ __forceinline__ int circle_mate(int r, int i) {
  constexpr int n1 = kJP - 1;
  if (i == n1) return r;
  if (i == r) return n1;
  return (2 * r - i + 2 * n1) % n1;
}

// Partner of index i in step k of a cross sweep: step k rotates the planes
// (i, kJW + (i + k) mod kJW), i < kJW, so kJW steps meet every pair of one
// column of each block once.
__device__ __forceinline__ int cross_mate(int k, int i) {
  static_assert((kJW & (kJW - 1)) == 0, "cross_mate: kJW a power of two");
  return i < kJW ? kJW + ((unsigned)(i + k) & (kJW - 1)) : ((unsigned)(i - kJW - k + 2 * kJW) & (kJW - 1));
}

// plane `slot` of step r: (p, q), p < q
__device__ __forceinline__ void step_plane(bool full, int r, int slot, int& p, int& q) {
  if (full) {
    p = slot == 0 ? r : min(circle_mate(r, (r + slot) % (kJP - 1)), (r + slot) % (kJP - 1));
    q = circle_mate(r, p);
  } else {
    p = slot;
    q = cross_mate(r, slot);
  }
}

// Rotation of the plane (p, q), p < q, that zeroes g_pq: c and s with
// column p of G J = c g_p - s g_q and column q = s g_p + c g_q.  t = tan of
// the angle is the smaller root of t^2 + 2 (a / b) t - 1 = 0, a = g_qq -
// g_pp, b = 2 g_pq: t = sign(a) b / (|a| + sqrt(a^2 + b^2)).  Any t close to
// it gives an exactly orthogonal rotation that nearly zeroes g_pq (the
// sweeps repeat until the off-diagonal is small), so t is formed with the
// hardware's approximate square root and reciprocal, after an exact scaling
// of a and b by a power of two; c = 1 / sqrt(1 + t^2) takes the hardware's
// reciprocal square root and two Newton steps (about one ulp), and s = c t,
// so that c^2 + s^2 = 1 to rounding.
__device__ __forceinline__ void jacobi_rot(double gpp, double gqq, double gpq, double& c, double& s) {
  c = 1.0;
  s = 0.0;
  if (!(fabs(gpq) > 1e-300 && gpq * gpq > 0x1p-104 * fabs(gpp * gqq))) return;
  double a = gqq - gpp, b = 2.0 * gpq;
  const int ex = ilogb(fmax(fabs(a), fabs(b)));
  a = ldexp(a, -ex);
  b = ldexp(b, -ex);
  const double hyp = __builtin_amdgcn_sqrt(fma(a, a, b * b));
  const double tn = (a >= 0.0 ? b : -b) * __builtin_amdgcn_rcp(fabs(a) + hyp);
  const double x = fma(tn, tn, 1.0);
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-(x * y), y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  c = y;
  s = y * tn;
}

// Per pair: G = the partials summed in chunk order; the measure (sq_part,
// largest e_pq against skip); then kJW disjoint rotations per step, G <- J^T
// G J and Q <- Q J, one thread per entry: with `full` (the first round of an
// outer sweep) a cyclic sweep over all kJP indices (kJP - 1 steps), else a
// cross sweep (kJW steps: every pair of one column from each block once, the
// blocks' own pairs having had their turn in the sweep's first round, where
// every block meets its partner in a full sweep).  One
// barrier per step: thread k < kJW first forms the three entries of the next
// G that the next step's k-th plane needs and computes that rotation
// (rotations double-buffered by step parity), then, like every thread, its
// entry of the next G and Q with the step's rotations.  Q to qbuf
// (row-major) and flag[pair] = 0, or flag = 1 (skip: X and V keep the
// pair's columns).
constexpr int kJRT = kJP * kJP;  // threads of k_jac_rot (one per entry)
// MEAS: only the sums and the measure (a measurement pass: no rotation);
// with `blocks` (the pass's first round, where every block sits in exactly
// one pair) the entries within each block count too, so that the pass sums
// every off-diagonal entry of the state once.
template <bool FULL, bool MEAS = false>
__global__ void __launch_bounds__(kJRT) k_jac_rot(const double* __restrict__ gpart, int nchunk, double d2,
                                                   double skip, double* __restrict__ sq_part,
                                                   double* __restrict__ qbuf, int* __restrict__ flag,
                                                   int blocks = 0) {
  __shared__ double G[2][kJP][kJP + 1];
  __shared__ double Q[2][kJP][kJP + 1];
  __shared__ double cs[2][kJP], sn[2][kJP];  // per step parity and index: its plane's c and signed s
  __shared__ double wmax[kJRT / kWave], wsq[kJRT / kWave];
  const int pair = blockIdx.x, tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
  const int i = tid / kJP, j = tid % kJP;
  const double* gp = gpart + (long long)pair * nchunk * (kJP * kJP);
  {
    double v[kJMaxChunks];
#pragma unroll
    for (int c = 0; c < kJMaxChunks; ++c) v[c] = c < nchunk ? gp[(long long)c * (kJP * kJP) + tid] : 0.0;
    double g = 0.0;
#pragma unroll
    for (int c = 0; c < kJMaxChunks; ++c) g += v[c];
    G[0][i][j] = g;
    Q[0][i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  double mx = 0.0, sq = 0.0;
  if (i < j) {
    const double d = sqrt((G[0][i][i] + d2) * (G[0][j][j] + d2));
    const double v = d > 0.0 ? fabs(G[0][i][j]) / d : 0.0;
    mx = v;
    if ((i < kJW && j >= kJW) || (MEAS && blocks)) sq = v * v;
  }
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    mx = fmax(mx, __shfl_xor(mx, o, kWave));
    sq += __shfl_xor(sq, o, kWave);
  }
  if (lane == 0) {
    wmax[wave] = mx;
    wsq[wave] = sq;
  }
  // step 0's rotations from G itself
  if (!MEAS && tid < kJW) {
    int p, q;
    step_plane(FULL, 0, tid, p, q);
    double c, s;
    jacobi_rot(G[0][p][p], G[0][q][q], G[0][p][q], c, s);
    cs[0][p] = cs[0][q] = c;
    sn[0][p] = -s;
    sn[0][q] = s;
  }
  __syncthreads();
  double block_off = 0.0, block_sq = 0.0;
#pragma unroll
  for (int w = 0; w < kJRT / kWave; ++w) {
    block_off = fmax(block_off, wmax[w]);
    block_sq += wsq[w];
  }
  if (tid == 0) sq_part[pair] = block_sq;
  if (MEAS) return;
  if (block_off <= skip) {  // uniform
    if (tid == 0) flag[pair] = 1;
    return;
  }
  constexpr bool fl = FULL;
  const int steps = fl ? kJP - 1 : kJW;
  auto mate = [&](int r, int x) { return fl ? circle_mate(r, x) : cross_mate(r, x); };
  int cur = 0;
  for (int r = 0; r < steps; ++r) {
    const int nx = cur ^ 1, par = r & 1;
    if (tid < kJW && r + 1 < steps) {
      // the next step's plane tid: its entries of the next G, then its rotation
      int p, q;
      step_plane(fl, r + 1, tid, p, q);
      auto next = [&](int x, int y) {
        const int mx_ = mate(r, x), my = mate(r, y);
        const double cx = cs[par][x], sx = sn[par][x], cy = cs[par][y], sy = sn[par][y];
        const double gxy = cy * G[cur][x][y] + sy * G[cur][x][my];
        const double gmy = cy * G[cur][mx_][y] + sy * G[cur][mx_][my];
        return cx * gxy + sx * gmy;
      };
      const double gpp = next(p, p), gqq = next(q, q), gpq = next(p, q);
      double c, s;
      jacobi_rot(gpp, gqq, gpq, c, s);
      cs[par ^ 1][p] = cs[par ^ 1][q] = c;
      sn[par ^ 1][p] = -s;
      sn[par ^ 1][q] = s;
    }
    {
      // entry (i, j) of J^T G J and of Q J for this step's planes
      const int mi = mate(r, i), mj = mate(r, j);
      const double ci = cs[par][i], si = sn[par][i], cj = cs[par][j], sj = sn[par][j];
      const double gij = cj * G[cur][i][j] + sj * G[cur][i][mj];
      const double gmj = cj * G[cur][mi][j] + sj * G[cur][mi][mj];
      G[nx][i][j] = ci * gij + si * gmj;
      Q[nx][i][j] = cj * Q[cur][i][j] + sj * Q[cur][i][mj];
    }
    cur = nx;
    __syncthreads();
  }
  qbuf[(long long)pair * (kJP * kJP) + tid] = Q[cur][i][j];
  if (tid == 0) flag[pair] = 0;
}

// Rows [kJARows blockIdx.x + 16 kJAJ wave, + 16 kJAJ) of X (blockIdx.z = 0)
// or V (1), the pair's columns, times Q: D = Q^T X_rows^T on the FP64 16x16x4 MFMA (A lane
// (i, q) = Q[k + q][16 It + i] from LDS, B lane (i, q) = X[row0 + i][col(k + q)],
// D lane (i, q) register r = the new X[row0 + i][col(16 It + q + 4r)]).  All of
// the wave's loads precede its stores, and no other wave touches these rows
// and columns, so the update is in place.
__global__ void __launch_bounds__(kJT) k_jac_apply(double* __restrict__ X, long long ldx, int xrows,
                                                    double* __restrict__ V, long long ldv, int vrows, int nblk,
                                                    int round, const double* __restrict__ qbuf,
                                                    const int* __restrict__ flag) {
  constexpr int NI = kJP / 16, KS = kJP / 4, NJ = kJAJ;
  __shared__ double Qs[kJP][kJP + 1];
  const int pair = blockIdx.y;
  if (flag[pair]) return;  // uniform
  double* M = blockIdx.z ? V : X;
  const long long ld = blockIdx.z ? ldv : ldx;
  const int rows = blockIdx.z ? vrows : xrows;
  if ((long long)blockIdx.x * kJARows >= rows) return;  // uniform
  int a, b;
  pair_of(round, nblk, pair, a, b);
  const double* qp = qbuf + (long long)pair * (kJP * kJP);
  for (int e = threadIdx.x; e < kJP * kJP; e += kJT) Qs[e / kJP][e % kJP] = qp[e];
  __syncthreads();
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave, li = lane % 16, lq = lane / 16;
  const int r0 = blockIdx.x * kJARows + wave * (16 * NJ);
  if (r0 >= rows) return;  // no barrier follows
  double xv[NJ][KS];
#pragma unroll
  for (int jt = 0; jt < NJ; ++jt)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int r = r0 + 16 * jt + li;
      xv[jt][ks] = r < rows ? M[(long long)pair_col(a, b, 4 * ks + lq) * ld + r] : 0.0;
    }
  f64x4_t acc[NI][NJ];
#pragma unroll
  for (int it = 0; it < NI; ++it)
#pragma unroll
    for (int jt = 0; jt < NJ; ++jt) acc[it][jt] = (f64x4_t){0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int ks = 0; ks < KS; ++ks)
#pragma unroll
    for (int it = 0; it < NI; ++it) {
      const double qa = Qs[4 * ks + lq][16 * it + li];
#pragma unroll
      for (int jt = 0; jt < NJ; ++jt)
        acc[it][jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(qa, xv[jt][ks], acc[it][jt], 0, 0, 0);
    }
#pragma unroll
  for (int it = 0; it < NI; ++it)
#pragma unroll
    for (int jt = 0; jt < NJ; ++jt) {
      const int r = r0 + 16 * jt + li;
      if (r < rows) {
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) M[(long long)pair_col(a, b, 16 * it + lq + 4 * rr) * ld + r] = acc[it][jt][rr];
      }
    }
}

__global__ void k_col_norms(const double* X, long long ldx, int rows, int ncols, double* out) {
  const int c = blockIdx.x;
  if (c >= ncols) return;
  double s = 0.0;
  for (int r = threadIdx.x; r < rows; r += kBlock) {
    const double v = X[(long long)r + (long long)c * ldx];
    s += v * v;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) out[c] = sqrt(s);
}

// out[0] = sum of part[0..count) in a fixed order (thread-strided sums, a
// shuffle tree, the waves in order): the same value on every run.
__global__ void __launch_bounds__(kBlock) k_sum_fixed(const double* part, int count, double* out) {
  double v = 0.0;
  for (int i = threadIdx.x; i < count; i += kBlock) v += part[i];
  v = block_sum(v);
  if (threadIdx.x == 0) out[0] = v;
}

// A measurement pass runs when the last two sweeps' measures extrapolate to
// at most this multiple of the stopping level.
constexpr double kJacMeasureFactor = 2.0;

// Row chunks of the Gram launch: about 1024 workgroups per round, chunks of
// at least 64 rows (a multiple of 16), at most kJMaxChunks.
static void jacobi_chunks(int rows, int npairs, int& nchunk, int& rpc) {
  int want = (1024 + npairs - 1) / npairs;
  want = std::max(1, std::min(std::min(want, kJMaxChunks), (rows + 63) / 64));
  rpc = ((rows + want - 1) / want + 15) / 16 * 16;
  nchunk = std::max(1, (rows + rpc - 1) / rpc);
}

struct JacWork {
  double *sq_part, *sum, *gpart, *qbuf;
  int* flag;
};

static JacWork carve_jacobi(double* w, int rows, int npad) {
  const long long nblk = npad / kJW, npairs = nblk / 2, rounds = nblk - 1;
  JacWork j;
  j.sq_part = w;
  j.sum = w + rounds * npairs;
  j.gpart = j.sum + 1;
  j.qbuf = j.gpart + npairs * (long long)kJMaxChunks * kJP * kJP;
  j.flag = (int*)(j.qbuf + npairs * (long long)kJP * kJP);
  (void)rows;
  return j;
}

int jacobi_svd(double* X, long long ldx, int n, int npad, double* Vm, long long ldv, double* sigma, double* work,
               double delta2, double tol_f, double skip, int max_sweeps, hipStream_t s) {
  // X: n x npad (columns n..npad-1 zero), Vm: npad x npad, set by the caller.
  APL_REQUIRE(npad % kJP == 0 && npad >= kJP, "jacobi_svd: npad must be a positive multiple of the pair width");
  const int nblk = npad / kJW;
  const int npairs = nblk / 2, rounds = nblk - 1;
  int nchunk, rpc;
  jacobi_chunks(n, npairs, nchunk, rpc);
  const JacWork jw = carve_jacobi(work, n, npad);
  const int arows = std::max(n, npad);
  const dim3 ga(ceil_div(arows, kJARows), npairs, 2);
  // the fixed-order sum of the per-pair measures of the last pass
  auto read_measure = [&]() {
    hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(kBlock), 0, s, (const double*)jw.sq_part, rounds * npairs, jw.sum);
    double sum_sq = 0.0;
    APL_HIP(hipMemcpyAsync(&sum_sq, jw.sum, sizeof(sum_sq), hipMemcpyDeviceToHost, s));
    APL_HIP(hipStreamSynchronize(s));
    return std::sqrt(2.0 * sum_sq);
  };
  double prev_eps = INFINITY;
  int sweeps = 0;
  for (; sweeps < max_sweeps; ++sweeps) {
    for (int r = 0; r < rounds; ++r) {
      hipLaunchKernelGGL(k_jac_gram, dim3(nchunk, npairs), dim3(kJT), 0, s, (const double*)X, ldx, n, nblk, r, rpc,
                         nchunk, jw.gpart);
      if (r == 0)
        hipLaunchKernelGGL(k_jac_rot<true>, dim3(npairs), dim3(kJRT), 0, s, (const double*)jw.gpart, nchunk, delta2,
                           skip, jw.sq_part + (long long)r * npairs, jw.qbuf, jw.flag);
      else
        hipLaunchKernelGGL(k_jac_rot<false>, dim3(npairs), dim3(kJRT), 0, s, (const double*)jw.gpart, nchunk,
                           delta2, skip, jw.sq_part + (long long)r * npairs, jw.qbuf, jw.flag);
      hipLaunchKernelGGL(k_jac_apply, ga, dim3(kJT), 0, s, X, ldx, n, Vm, ldv, npad, nblk, r,
                         (const double*)jw.qbuf, (const int*)jw.flag);
    }
    // Frobenius norm of the damped off-diagonal (both triangles) as the sweep saw it
    const double eps = read_measure();
    if (eps <= tol_f) {
      ++sweeps;
      break;
    }
    // When the measures of the last two sweeps extrapolate (geometrically)
    // to the stopping level, measure the state this sweep left, pair by
    // pair without rotating (every off-diagonal entry once, the entries
    // within blocks included): if that meets the test, the next sweep is not
    // needed (its rotations would only refine a state that already passes).
    if (sweeps >= 1 && eps * (eps / prev_eps) <= kJacMeasureFactor * tol_f) {
      for (int r = 0; r < rounds; ++r) {
        hipLaunchKernelGGL(k_jac_gram, dim3(nchunk, npairs), dim3(kJT), 0, s, (const double*)X, ldx, n, nblk, r,
                           rpc, nchunk, jw.gpart);
        hipLaunchKernelGGL((k_jac_rot<false, true>), dim3(npairs), dim3(kJRT), 0, s, (const double*)jw.gpart,
                           nchunk, delta2, skip, jw.sq_part + (long long)r * npairs, jw.qbuf, jw.flag, r == 0 ? 1 : 0);
      }
      if (read_measure() <= tol_f) {
        ++sweeps;
        break;
      }
    }
    prev_eps = eps;
  }
  hipLaunchKernelGGL(k_col_norms, dim3(n), dim3(kBlock), 0, s, (const double*)X, ldx, n, n, sigma);
  return sweeps;
}

long long jacobi_work_words(int npad) {
  const long long nblk = npad / kJW, npairs = nblk / 2, rounds = nblk - 1;
  return rounds * npairs + 1 + npairs * (long long)kJMaxChunks * kJP * kJP + npairs * (long long)kJP * kJP +
         (npairs + 1) / 2 + 1;
}

int jacobi_block_width() { return kJW; }

// ============================================================== preconditioner scalars
// d_i = target / sqrt(sigma_i^2 + delta^2) - 1, with target = sqrt(min sigma^2 + delta^2);
// info[0] = min sigma, info[1] = max sigma, info[2] = target, info[3] = pnorm.
__global__ void k_precond_scalars(const double* sigma, int l, double delta, double* d, double* info) {
  __shared__ double smin, smax;
  if (threadIdx.x == 0) {
    double a = INFINITY, b = 0.0;
    for (int i = 0; i < l; ++i) {
      a = fmin(a, sigma[i]);
      b = fmax(b, sigma[i]);
    }
    smin = a;
    smax = b;
  }
  __syncthreads();
  const double target = sqrt(smin * smin + delta * delta);
  for (int i = threadIdx.x; i < l; i += kBlock) d[i] = target / sqrt(sigma[i] * sigma[i] + delta * delta) - 1.0;
  if (threadIdx.x == 0) {
    info[0] = smin;
    info[1] = smax;
    info[2] = target;
    info[3] = fmax(1.0, sqrt(smax * smax + delta * delta) / target);
  }
}

void precond_scalars(const double* sigma, int l, double delta, double* d, double* info, hipStream_t s) {
  hipLaunchKernelGGL(k_precond_scalars, dim3(1), dim3(kBlock), 0, s, sigma, l, delta, d, info);
}

// rho = 10 sqrt(2/pi) max_i ||EW(:, i)||  (EW = E_row W, s x r column-major).
__global__ void k_rho(const double* EW, int s_rows, int r, double* out) {
  __shared__ double norms[64];
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  for (int c = w; c < r; c += kBlock / kWave) {
    double acc = 0.0;
    for (int h = l; h < s_rows; h += kWave) acc += EW[h + (long long)c * s_rows] * EW[h + (long long)c * s_rows];
    acc = wave_sum(acc);
    if (l == 0) norms[c] = sqrt(acc);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double mx = 0.0;
    for (int c = 0; c < r; ++c) mx = fmax(mx, norms[c]);
    out[0] = 10.0 * sqrt(2.0 / M_PI) * mx;
  }
}

void rho_from_ew(const double* EW, int s_rows, int r, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_rho, dim3(1), dim3(kBlock), 0, s, EW, s_rows, r, out);
}

// Copy a column-major block (rows x cols) with scaling: dst = alpha * src.
__global__ void k_copy_block(const double* src, long long lds, double* dst, long long ldd, int rows, int cols,
                             double alpha) {
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  const int j = blockIdx.y;
  if (i < rows && j < cols) dst[i + j * ldd] = alpha * src[i + j * lds];
}

void copy_block(const double* src, long long lds, double* dst, long long ldd, int rows, int cols, double alpha,
                hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL(k_copy_block, dim3(ceil_div(rows, kBlock), cols), dim3(kBlock), 0, s, src, lds, dst, ldd,
                     rows, cols, alpha);
}

__global__ void k_add_block(const double* src, long long lds, double* dst, long long ldd, int rows, int cols) {
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  const int j = blockIdx.y;
  if (i < rows && j < cols) dst[i + j * ldd] += src[i + j * lds];
}

void add_block(const double* src, long long lds, double* dst, long long ldd, int rows, int cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL(k_add_block, dim3(ceil_div(rows, kBlock), cols), dim3(kBlock), 0, s, src, lds, dst, ldd, rows,
                     cols);
}

// C = alpha * sum_p W_p + beta * C  (W_p: m x n column-major, summed in order)
__global__ void k_splitk_reduce(const double* W, int parts, long long m, long long n, double alpha, double beta,
                                double* C, long long ldc) {
  const long long mn = m * n;
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < mn; e += (long long)gridDim.x * kBlock) {
    double acc = 0.0;
    for (int p = 0; p < parts; ++p) acc += W[(long long)p * mn + e];
    const long long i = e % m, j = e / m;
    double* out = C + i + j * ldc;
    *out = beta == 0.0 ? alpha * acc : alpha * acc + beta * *out;
  }
}

void splitk_reduce(const double* W, int parts, long long m, long long n, double alpha, double beta, double* C,
                   long long ldc, hipStream_t s) {
  unsigned g = ceil_div(m * n, kBlock);
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_splitk_reduce, dim3(g), dim3(kBlock), 0, s, W, parts, m, n, alpha, beta, C, ldc);
}

__global__ void k_set_identity(double* X, long long ld, int n) {
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  const int j = blockIdx.y;
  if (i < n) X[i + j * ld] = (i == j) ? 1.0 : 0.0;
}

void set_identity(double* X, long long ld, int n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_set_identity, dim3(ceil_div(n, kBlock), n), dim3(kBlock), 0, s, X, ld, n);
}

__global__ void k_add_diag(double* X, long long ld, int n, double v) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) X[i + (long long)i * ld] += v;
}

void add_diag(double* X, long long ld, int n, double v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_add_diag, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, X, ld, n, v);
}

// Column-major dst = src^T (n x n): dst[i n + j] = src[j lds + i], 32 x 32
// tiles through LDS so that both the loads and the stores are coalesced.
__global__ void __launch_bounds__(kBlock) k_transpose(const double* src, long long lds, double* dst, int n) {
  __shared__ double tile[32][33];
  const int bi = blockIdx.y * 32, bj = blockIdx.x * 32;
  const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
  for (int r = ty; r < 32; r += kBlock / 32) {
    const int i = bi + tx, j = bj + r;
    tile[tx][r] = (i < n && j < n) ? src[(long long)j * lds + i] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += kBlock / 32) {
    const int i = bi + r, j = bj + tx;
    if (i < n && j < n) dst[(long long)i * n + j] = tile[r][tx];
  }
}

void transpose_square(const double* src, long long lds, double* dst, int n, hipStream_t s) {
  if (n <= 0) return;
  dim3 g(ceil_div(n, 32), ceil_div(n, 32));
  hipLaunchKernelGGL(k_transpose, g, dim3(kBlock), 0, s, src, lds, dst, n);
}

// ---------------------------------------------------------------- column scaling
__global__ void k_scale_cols(const double* X, long long ld, int rows, int cols, const double* d, double* out) {
  const long long total = (long long)rows * cols;
  for (long long t = (long long)blockIdx.x * kBlock + threadIdx.x; t < total; t += (long long)gridDim.x * kBlock) {
    const long long i = t % rows, j = t / rows;
    out[i + j * ld] = X[i + j * ld] * d[j];
  }
}

void scale_cols(const double* X, long long ld, int rows, int cols, const double* d, double* out, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  long long g = ((long long)rows * cols + kBlock - 1) / kBlock;
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_scale_cols, dim3((unsigned)g), dim3(kBlock), 0, s, X, ld, rows, cols, d, out);
}

// ---------------------------------------------------------------- FP32 copies
__global__ void k_to_f32(const double* src, long long lds, float* dst, long long ldd, long long rows, long long cols) {
  const long long total = rows * cols;
  for (long long t = (long long)blockIdx.x * kBlock + threadIdx.x; t < total; t += (long long)gridDim.x * kBlock) {
    const long long i = t / cols, j = t % cols;
    dst[i * ldd + j] = (float)src[i * lds + j];
  }
}

void to_f32(const double* src, long long lds, float* dst, long long ldd, long long rows, long long cols,
            hipStream_t s) {
  if (rows <= 0 || cols <= 0) return;
  long long g = (rows * cols + kBlock - 1) / kBlock;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_to_f32, dim3((unsigned)g), dim3(kBlock), 0, s, src, lds, dst, ldd, rows, cols);
}

// ---------------------------------------------------------------- adjoint helpers
__global__ void k_sub_cols(const double* B, long long ldb, const double* AX, long long ldax, double* R, long long ldr,
                           long long m, int k) {
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  const int q = blockIdx.y;
  if (i < m && q < k) R[q * ldr + i] = B[q * ldb + i] - AX[q * ldax + i];
}

void sub_cols(const double* B, long long ldb, const double* AX, long long ldax, double* R, long long ldr, long long m,
              int k, hipStream_t s) {
  if (m <= 0 || k <= 0) return;
  hipLaunchKernelGGL(k_sub_cols, dim3(ceil_div(m, kBlock), k), dim3(kBlock), 0, s, B, ldb, AX, ldax, R, ldr, m, k);
}

// One thread per row: the row's non-zeros, each a k-term sum.
__global__ void k_grad_csr(const int* rp, const int* ci, long long m, int k, const double* R, long long ldr,
                           const double* Z, long long ldz, const double* AZ, long long ldaz, const double* X,
                           long long ldx, double* dA) {
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (i >= m) return;
  for (int e = rp[i]; e < rp[i + 1]; ++e) {
    const long long j = ci[e];
    double acc = 0.0;
    for (int q = 0; q < k; ++q) acc += R[q * ldr + i] * Z[q * ldz + j] - AZ[q * ldaz + i] * X[q * ldx + j];
    dA[e] = acc;
  }
}

void grad_csr(const int* row_ptr, const int* col_idx, long long m, int k, const double* R, long long ldr,
              const double* Z, long long ldz, const double* AZ, long long ldaz, const double* X, long long ldx,
              double* dA, hipStream_t s) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_grad_csr, dim3(ceil_div(m, kBlock)), dim3(kBlock), 0, s, row_ptr, col_idx, m, k, R, ldr, Z, ldz,
                     AZ, ldaz, X, ldx, dA);
}

}  // namespace aplicur
