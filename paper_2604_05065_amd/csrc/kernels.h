// Launch functions of the APLICUR HIP kernels (host side declarations).
#pragma once

#include "common.h"

namespace aplicur {

// ---- set-up: random stream, CSR transpose, sketch (kern_sketch.hip)
void launch_gen_sketch(uint64_t seed, int s, long long m, int xi, uint16_t* rows,
                       uint8_t* negmask, hipStream_t st);
int check_csr(const int* row_ptr, const int* col_idx, long long m, long long n, long long nnz, int* bad_dev,
              hipStream_t st);
void launch_gen_probes(uint64_t seed, long long n, int r, double* W, hipStream_t st);
template <class T>
void launch_csr_transpose(const int* row_ptr, const int* col_idx, const T* val, long long m,
                          long long n, long long nnz, int* t_ptr, int* t_idx, T* t_val,
                          int* scratch_n, hipStream_t st);
template <class T>
void launch_sketch_csr(const int* t_ptr, const int* t_idx, const T* t_val, long long n, int s,
                       int xi, const uint16_t* rows, const uint8_t* negmask, double* Y,
                       hipStream_t st);
int sketch_dense_chunks(long long m, long long n);
template <class T>
void launch_sketch_dense(const T* A, long long m, long long n, long long ld, int s, int xi,
                         const uint16_t* rows, const uint8_t* negmask, double* Y, double* part,
                         int chunks, hipStream_t st);

// ---- Golub-Kahan / LSQR (kern_gk.hip)
// Operator description shared by the products: CSR (row_ptr/col_idx/val and
// the transpose t_ptr/t_idx/t_val) or dense row-major (val, ld).
struct OpDesc {
  int csr;            // 1: CSR, 0: dense row-major
  int f64;            // 1: values are double, 0: float
  long long m, n, ld, nnz;
  const int *rb, *t_rb;          // row blocks of the CSR-stream products (A, A^T)
  const int *row_ptr, *col_idx;  // CSR of A
  const void* val;
  const int *t_ptr, *t_idx;      // CSR of A^T
  const void* t_val;
  int group;          // lanes per CSR row (A), power of two
  int t_group;        // lanes per CSR row (A^T)
  double* part;       // partial buffer for dense A^T (chunks x n)
  int chunks;         // row chunks of the dense A^T product
};

// Preconditioner in explicit form: P^{-1} z = z + V (d .* (V^T z)), V row-major n x ell.
struct PrecDesc {
  int ell;
  long long ldv;
  const double* V;
  const double* d;
  double* part;   // chunks x ell
  int chunks;
  double* c;      // ell
};

// Work vectors of one right-hand side (precision V = double or float).
template <class V>
struct GKVecs {
  V *u_top, *u_bot, *v, *w, *y, *t, *g;
};

// Partial-sum buffers of the fence-free reductions (alpha: norms of v, beta:
// norms of u) and the number of partials the last producer wrote.
struct GKWork {
  double* alpha_part;
  double* beta_part;
  unsigned alpha_count, beta_count;
};

// st points to the two state slots (see kern_gk.hip).
template <class V>
void gk_iteration(const OpDesc& A, const PrecDesc* P, GKVecs<V> vec, GKState* st, GKWork& wk, hipStream_t s);
// Phase start: r = [b - A x; bot_scale b_bot - delta x] in FP64 (b or b_bot may be
// null = 0; x null = 0), beta_1 = ||r||, v_1 = P^{-T} A_mu^T u_1 (alpha finished by
// the first kernel of the first iteration).
template <class V>
void gk_phase_init(const OpDesc& A, const PrecDesc* P, const double* b, const double* b_bot, double bot_scale,
                   const double* x, GKVecs<V> vec, double* r_top64, double* r_bot64, GKState* st, GKWork& wk,
                   hipStream_t s);
// Phase end: x += P^{-1} y.
template <class V>
void gk_phase_finish(const OpDesc& A, const PrecDesc* P, GKVecs<V> vec, double* x, GKState* st, hipStream_t s);
// ||A_mu^T r||^2 -> st[0].h2 for r = [b - A x; bot_scale b_bot - delta x].
void gk_normal_residual(const OpDesc& A, const double* b, const double* b_bot, double bot_scale, const double* x,
                        GKVecs<double> vec, GKState* st, GKWork& wk, hipStream_t s);
void op_atb_norm2(const OpDesc& A, const double* b, double* tmp_n, GKState* st, GKWork& wk, hipStream_t s);
void op_norm(const OpDesc& A, const double* b, double* tmp_m, GKState* st, GKWork& wk, hipStream_t s);
void op_matvec(const OpDesc& A, int trans, const double* x, double* y, GKState* st, GKWork& wk, hipStream_t s);
template <class V>
void fill_zero(V* p, long long n, hipStream_t s);
int stream_blocks(long long nnz);
void build_row_blocks(const int* rp, long long m, long long nnz, int* rb, hipStream_t s);

}  // namespace aplicur
