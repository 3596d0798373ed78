// Host declarations of the CUR / factorisation kernels (kern_factor.hip).
#pragma once

#include <climits>
#include <cstring>

#include "kernels.h"

namespace aplicur {

using AMat = OpDesc;

// Scratch of the pivot search (sized for the tallest matrix searched).
struct FactorWork {
  int lupp_rows;
  int *pos, *row_at;
  double* pv;
  int *pp, *pi;
  void* lupp_state;
  unsigned* counter;
  double* lupp_g;  // pivot rows of a panel, kLuppNB x (sketch columns)
};

// First k partial-pivoting pivots of the column-major r x c matrix X (X is
// overwritten).  piv[0..keff) receives original row indices; read keff with
// lupp_read_keff (synchronises the stream).
void lupp_pivots(double* X, int r, int c, long long ld, int k, int* piv, FactorWork& fw, hipStream_t s);
int lupp_read_keff(FactorWork& fw, hipStream_t s);
// Pieces of the same pivot sequence computed panel by panel (the host then
// updates the trailing columns with a TRSM and a GEMM): lupp_begin (candidates
// of column 0), lupp_step (pivot q; eliminates columns up to cend), lupp_cand
// (candidates of column col after the trailing update), lupp_gather (the
// panel's pivot rows, G = X(piv[q0..q0+nb), q0..q0+w), column-major nb x w).
void lupp_begin(double* X, int r, int k, FactorWork& fw, hipStream_t s);
void lupp_step(double* X, int r, int c, int cend, long long ld, int q, int k, int* piv, FactorWork& fw,
               hipStream_t s);
void lupp_cand(const double* X, int r, long long ld, int col, FactorWork& fw, hipStream_t s);
void lupp_gather(const double* X, int r, long long ld, const int* piv, int q0, int nb, int w, double* G,
                 hipStream_t s);

void gather_cols(const AMat& A, const int* J, int k, double* out, long long ld_out, hipStream_t s);
void gather_rows(const AMat& A, const int* I, int k, double* out, long long ld_out, hipStream_t s);
void gather_sub_rows(const double* X, long long ldx, const int* rows, int nr, int ncols, double* out,
                     long long ldo, hipStream_t s);
void gather_y_cols(const double* Y, long long n, int s_rows, const int* J, int k, double* out, long long ldo,
                   hipStream_t s);
void zero_rows(double* X, long long ldx, const int* rows, int nr, int ncols, hipStream_t s);
void fill(double* X, long long n, double v, hipStream_t s);
void copy_block(const double* src, long long lds, double* dst, long long ldd, int rows, int cols, double alpha,
                hipStream_t s);
void splitk_reduce(const double* W, int parts, long long m, long long n, double alpha, double beta, double* C,
                   long long ldc, hipStream_t s);
void set_identity(double* X, long long ld, int n, hipStream_t s);
// X(i, i) += v for i < n (column-major, ld).
void add_diag(double* X, long long ld, int n, double v, hipStream_t s);
// out (column-major, ld) = X diag(d): column j scaled by d[j].
void scale_cols(const double* X, long long ld, int rows, int cols, const double* d, double* out, hipStream_t s);
// dst (rows x cols, row-major, ldd) = (float) src (row-major, lds); contiguous when rows = 1.
void to_f32(const double* src, long long lds, float* dst, long long ldd, long long rows, long long cols,
            hipStream_t s);
// R (m x k, ldr) = B - AX (column-major).
void sub_cols(const double* B, long long ldb, const double* AX, long long ldax, double* R, long long ldr, long long m,
              int k, hipStream_t s);
// Gradient on a CSR pattern: dA_e = sum_q R(i,q) Z(j,q) - AZ(i,q) X(j,q) for every
// non-zero e = (i, j), column-major R (m x k), Z, X (n x k), AZ (m x k).
void grad_csr(const int* row_ptr, const int* col_idx, long long m, int k, const double* R, long long ldr,
              const double* Z, long long ldz, const double* AZ, long long ldaz, const double* X, long long ldx,
              double* dA, hipStream_t s);
// dst (n x n, ld n) = src^T (src n x n, ld lds).
void transpose_square(const double* src, long long lds, double* dst, int n, hipStream_t s);
void add_block(const double* src, long long lds, double* dst, long long ldd, int rows, int cols, hipStream_t s);

// Pieces of the blocked Cholesky / LU of small dense matrices (column-major):
// block width kFNB, at most kFMaxRows rows in an LU panel.
constexpr int kFNB = 64;
constexpr int kFMaxRows = 288;
void potrf_diag(double* G, long long ld, int nb, int j0, int* status, hipStream_t s);
void lu_panel(double* A, long long ld, int k, int j0, int w, int* piv, int* status, hipStream_t s);
void laswp(double* A, long long ld, int ncols, int c0, int c1, const int* piv, int j0, int w, hipStream_t s);
void zero_lower(double* G, long long ld, int k, hipStream_t s);

int jacobi_block_width();
// One-sided block Jacobi SVD of X (n x npad, column-major; columns n.. zero):
// X <- X V, Vm <- Vm V (Vm holds the starting orthogonal basis on entry,
// npad x npad; npad a multiple of 2 jacobi_block_width()), sigma[i] =
// ||X(:, i)|| for i < n.  Sweeps end once the Frobenius norm of the
// off-diagonal of the damped, scaled Gram matrix, e_pq = |g_pq| / sqrt((g_pp
// + delta2)(g_qq + delta2)), summed as the sweep met each block pair, is at
// most tol_f; a block pair with every e_pq <= skip is not rotated.  work:
// jacobi_work_words(npad) device doubles of scratch (per pair and round the
// partial sums of the stopping test, summed in a fixed order so that the
// sweep count does not depend on the order in which workgroups finish; the
// pairs' partial Gram matrices and rotations).  Returns the number of sweeps.
int jacobi_svd(double* X, long long ldx, int n, int npad, double* Vm, long long ldv, double* sigma, double* work,
               double delta2, double tol_f, double skip, int max_sweeps, hipStream_t s);
long long jacobi_work_words(int npad);
void precond_scalars(const double* sigma, int l, double delta, double* d, double* info, hipStream_t s);
void rho_from_ew(const double* EW, int s_rows, int r, double* out, hipStream_t s);

}  // namespace aplicur
