// Dense FP64 BLAS-3 of the set-up (kern_blas.hip): the products and
// triangular solves of the CUR increments (Alg. 7), the core and its
// residual (Alg. 3 Part 1), augmentQR (Alg. 9), T_C and the preconditioner
// builds (Alg. 2 Part 2, Alg. 8).  Column-major operands with the usual
// BLAS argument conventions; everything is enqueued on the given stream.
#pragma once

#include "common.h"

namespace aplicur {

enum class Op { N, T };

// C (m x n) = alpha op(A) op(B) + beta C on the FP64 16x16x4 MFMA (128 x 128
// output tiles, 16-deep LDS stages).  beta = 0 does not read C.  When the
// output has few tiles and k is long, the k range is cut into chunks whose
// products go to `work` and are summed in chunk order; work_count is the
// capacity of `work` in doubles (chunks are reduced to fit; 0: none).  The
// chunk count depends on the shape and work_count only, so a caller that
// always passes the same scratch gets reproducible sums.
void dgemm(Op ta, Op tb, long long m, long long n, long long k, double alpha, const double* A, long long lda,
           const double* B, long long ldb, double beta, double* C, long long ldc, double* work, size_t work_count,
           hipStream_t s);
// doubles of `work` that dgemm would use for this shape (0: no k chunks)
size_t dgemm_work(Op ta, Op tb, long long m, long long n, long long k);

enum class Side { Left, Right };
enum class Uplo { Lower, Upper };
enum class Diag { NonUnit, Unit };

// B <- alpha op(T)^{-1} B (Left, B m x n, T m x m) or alpha B op(T)^{-1}
// (Right, T n x n): blocked substitution, 64 x 64 diagonal blocks of op(T)
// held in LDS (one thread per column (Left) or row (Right) of B), the
// off-diagonal blocks applied with dgemm.
void dtrsm(Side side, Uplo uplo, Op trans, Diag diag, long long m, long long n, double alpha, const double* T,
           long long ldt, double* B, long long ldb, double* work, size_t work_count, hipStream_t s);

// ||x||_2 of n doubles, summed in a fixed order; `tmp` holds at least
// kNrm2Parts + 1 doubles.  Synchronises the stream and returns the value.
constexpr int kNrm2Parts = 256;
double dnrm2(long long n, const double* x, double* tmp, hipStream_t s);

// Y (s x n, row-major) = S A for a row-major FP32 A (m x n, lda) and a
// column-major S (s x m), FP64 accumulation: the sketch S A of a Gaussian
// embedding.  bf16 = false: S rounded to FP32, FP32 MFMA products over
// 16-term chunks, each chunk sum added in FP64; bf16 = true: S and A rounded
// to BF16, BF16 MFMA products (exact in FP32) over 32-term chunks, chunk sums
// added in FP64.
void sketch_gemm_f32(const float* A, long long m, long long n, long long lda, const double* S, int s_rows,
                     double* Y, bool bf16, hipStream_t st);

}  // namespace aplicur
