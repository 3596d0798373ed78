// Blocked Golub-Kahan / LSQR for several right-hand sides of a dense A: the k
// columns keep independent LSQR recurrences (one GKState each, Sec. 2.2) and
// share the products, which become tall-skinny matrix products on MFMA.
//
// Layout: every block vector is row-major with kp columns (kp in {16, 32, 64},
// columns beyond k zero), so row j of the block is kp contiguous values.
// States: st[0..kp) is slot 0 and st[kp..2kp) slot 1, with the two-slot
// protocol of the single-column kernels (slot 0 written by the kernel that
// finishes alpha, slot 1 by the kernel that finishes beta).  A column whose
// state is stopped is left untouched by every kernel; columns that take no
// part in a phase start stopped.
#pragma once

#include "gk_scalar.h"
#include "kernels.h"

namespace aplicur {

// out[s][r][0..kp) = sum over the s-th chunk of the columns j of M[r][j] In[j][0..kp)
// (M row-major rows x cols with leading dimension ld, In row-major cols x kp).
// S chunks of the reduction index; the consumer sums the S planes in order.
// e0 / e1 (optional): events recording the product kernel's own start and end.
template <class TA, class TB, class ACC>
void rows_gemm(const TA* M, long long rows, long long cols, long long ld, const TB* In, int kp, ACC* out, int S,
               hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
int gemm_splits(long long rows, long long cols);  // S for a product with this many rows and columns

// At (n x m row-major, leading dimension ldt) = A^T for A m x n row-major.
template <class T>
void transpose_rect(const T* A, long long m, long long n, long long lda, T* At, long long ldt, hipStream_t s);

// Xp (rows x kp row-major) <-> columns c < k of X (column-major, ldx); pack zero-fills c >= k.
void pack_cols(const double* X, long long ldx, long long rows, int k, double* Xp, int kp, hipStream_t s);
void unpack_cols(const double* Xp, int kp, long long rows, int k, double* X, long long ldx, hipStream_t s);

// Dense operator of the blocked path: A and its transposed copy.
struct BlkOp;
// Y[:, c] (column-major, ldy) = (A or A^T) X[:, c] for c < k (X column-major,
// ldx).  prec 0: X packed into `in` (FP64, kp columns), FP64 accumulation of
// A's values; prec 1: X rounded to FP32, FP32 values and FP32 accumulation
// (the products of the FP32 phases; A an FP32 operator); prec 2: the BF16
// products (A with BF16 copies).  `part` holds the S product planes, summed
// in order in the product's type.
void blk_matmat(const BlkOp& A, bool trans, const double* X, long long ldx, int kp, int k, double* Y, long long ldy,
                int prec, void* in, void* part, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

struct BlkOp {
  const void* A;   // m x n row-major (ld)
  const void* At;  // n x m row-major (ldt)
  long long m, n, ld, ldt;
  int f64;         // values are double (else float)
  int Sm, Sn;      // splits of the A t and A^T u products
  // BF16 copies of A and A^T in the tiled layout of tile_bf16 (precision 2),
  // else null; when set, the FP32-vector products of the iteration use them
  const void* A16;
  const void* At16;
};

// BF16 copy of a row-major FP32 matrix (rows x cols, ld) in tiles of 32 rows
// x 64 columns (zero-padded), rounded to nearest even; dst holds
// bf16_tiled_elems(rows, cols) entries.
long long bf16_tiled_elems(long long rows, long long cols);
void tile_bf16(const float* src, long long rows, long long cols, long long ld, void* dst, hipStream_t s);
// out[s][r][0..kp) = the s-th chunk of sum_j T[r][j] In[j][0..kp) for a tiled
// BF16 T, FP32 In (cols x kp row-major) and FP32 accumulation (S chunks).
void rows_gemm16(const void* T, long long rows, long long cols, const float* In, int kp, float* out, int S,
                 hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

// Explicit P^{-1} z = z + V (d .* (V^T z)) with V (n x ell, ldv) and V^T (ell x n, ldvt), FP64.
// The explicit P for the blocked kernels, V diag(d) V^T: with W null, V (n x
// ell row-major) and V^T (ell x n row-major); with W set, the factored form
// Q_R W Q_R^T, V holding Q_R (n x ell row-major), Vt Q_R^T (ell x n
// row-major) and W = V_M diag(d) V_M^T (ell x ell, symmetric).
struct BlkPrec {
  const double *V, *Vt, *d, *W;
  long long ldv, ldvt;
  int ell, S1, S2, S3;  // splits of V^T z, of V c and of W c
};

template <class V>
struct BlkVecs {
  V *u_top, *u_bot, *v, *w, *y, *t, *g;  // m x kp (u_top) and n x kp
};

struct BlkWork {
  void *pm, *pn;        // product partials: Sm x m x kp and Sn x n x kp (V)
  double *pl, *pc, *pq; // P: S1 x ell x kp partials, ell x kp coefficients, S2 x n x kp partials
  double* pc2;          // P in factored form: W times the coefficients
  double *beta_part, *alpha_part;  // at most kBlkMaxGrid x kp each
  int beta_count, alpha_count;
  double* norm_part;    // column partials of the norm kernels (kBlkMaxGrid x kp)
};

constexpr int kBlkMaxGrid = 256;  // workgroups of the element-wise kernels (their partials are re-read)

// Phase start: r = [B - Ares X; bs Bbot - delta X] (FP64 with the values of
// Ares; X = 0 when x_zero) stored in the V vectors, then as the single-column
// phase start with the operator A (beta, the first A^T product and alpha).
// r_ready (V = double only): the top block of r as already formed (B - Ares X,
// or B when x_zero) with wk.pn holding the planes of A^T r_top from the same
// kernels; both products are then skipped and the results are unchanged.
template <class V>
void blk_phase_init(const BlkOp& Ares, const BlkOp& A, const BlkPrec* P, int kp, const double* B, const double* Bbot,
                    double bs, const double* X, bool x_zero, double delta, BlkVecs<V> vec, GKState* st, BlkWork& wk,
                    hipStream_t s, const double* r_ready = nullptr);
template <class V>
void blk_iteration(const BlkOp& A, const BlkPrec* P, int kp, double delta, BlkVecs<V> vec, GKState* st, BlkWork& wk,
                   hipStream_t s);
// X += P^{-1} Y (the last y update was applied by the kernel that stopped).
template <class V>
void blk_phase_finish(const BlkOp& A, const BlkPrec* P, int kp, BlkVecs<V> vec, double* X, BlkWork& wk,
                      hipStream_t s);

// Column partials (wk.norm_part, returns their count) of
//   mode 0: ||B||^2 (m rows);  mode 3: ||Bbot||^2 (n rows);  mode 1: ||A^T B||^2;
//   mode 2: ||A_mu^T r||^2 with r = [B - A X; bs Bbot - delta X]
//   (A_mu^T r = A^T r_top + delta r_bot).
// tmp_m (m x kp) and tmp_n (n x kp) are FP64 scratch.
// outv (optional, modes 1 and 2): the vector itself (A^T B, or A_mu^T r), n x kp.
int blk_norms(const BlkOp& A, int kp, int mode, const double* B, const double* Bbot, double bs, const double* X,
              double delta, double* tmp_m, double* tmp_n, BlkWork& wk, hipStream_t s, double* outv = nullptr);

}  // namespace aplicur
