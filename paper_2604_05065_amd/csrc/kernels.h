// Launch functions of the APLICUR HIP kernels (host side declarations).
#pragma once

#include <vector>

#include "common.h"

namespace aplicur {

// ---- set-up: random stream, CSR transpose, sketch (kern_sketch.hip)
void launch_gen_sketch(uint64_t seed, int s, long long m, int xi, uint16_t* rows,
                       uint8_t* negmask, hipStream_t st);
int check_csr(const int* row_ptr, const int* col_idx, long long m, long long n, long long nnz, int* bad_dev,
              hipStream_t st);
void launch_gen_probes(uint64_t seed, long long n, int r, double* W, hipStream_t st);
// Gaussian sketch S (s x m column-major, N(0, 1/s) entries, stream 3) and
// Y = S A for CSR A through the CSR of A^T (Y row-major s x n).
void launch_gen_gauss_sketch(uint64_t seed, int s, long long m, double* S, hipStream_t st);
template <class T>
void launch_sketch_gauss_csr(const int* t_ptr, const int* t_idx, const T* t_val, long long n, int s, const double* S,
                             double* Y, hipStream_t st);
void widen(const float* a, double* b, long long count, hipStream_t st);  // b = (double) a
template <class T>
void launch_csr_transpose(const int* row_ptr, const int* col_idx, const T* val, long long m,
                          long long n, long long nnz, int* t_ptr, int* t_idx, T* t_val,
                          int* scratch_n, hipStream_t st);
// CSR of R = A(I[0..ell), :) with FP64 values; returns nnz(R) (synchronises
// the stream); fails if it would exceed cap.
template <class T>
long long launch_gather_csr_rows(const int* row_ptr, const int* col_idx, const T* val, const int* I, int ell,
                                 int* r_ptr, int* r_idx, double* r_val, long long cap, int* scratch,
                                 hipStream_t st);
template <class T>
void launch_sketch_csr(const int* t_ptr, const int* t_idx, const T* t_val, long long n, int s,
                       int xi, const uint16_t* rows, const uint8_t* negmask, double* Y,
                       hipStream_t st);
// device scratch (bytes) of the dense sketch: the inverse of the embedding
size_t sketch_dense_scratch(long long m, int s, int xi);
template <class T>
void launch_sketch_dense(const T* A, long long m, long long n, long long ld, int s, int xi,
                         const uint16_t* rows, const uint8_t* negmask, double* Y, void* scratch,
                         hipStream_t st);

// ---- Golub-Kahan / LSQR (kern_gk.hip)
// Operator description shared by the products: CSR (row_ptr/col_idx/val and
// the transpose t_ptr/t_idx/t_val) or dense row-major (val, ld).
struct OpDesc {
  int csr;            // 1: CSR, 0: dense row-major
  int f64;            // 1: values are double, 0: float
  long long m, n, ld, nnz;
  const int *rb, *t_rb;          // row blocks of the CSR-stream products (A, A^T)
  int stream_t;                  // non-zeros per row block
  const int* lx_rb;              // row blocks of the LDS-resident A x kernel (null: not used)
  int lx_grid;                   // its workgroups
  // SELL-64 copy of A for the LDS-resident A x kernel (null: not built)
  const int *sell_off, *sell_w, *sell_ci;
  const void* sell_val;
  int sell_slices, sell_spw, sell_grid;  // slices, slices per workgroup, workgroups
  int sell_uw;                           // > 0: every slice has this width (offsets 64 uw s)
  long long sell_padded;                 // entries including padding
  const int *row_ptr, *col_idx;  // CSR of A
  const void* val;
  const int *t_ptr, *t_idx;      // CSR of A^T
  const void* t_val;
  int group;          // lanes per CSR row (A), power of two
  int t_group;        // lanes per CSR row (A^T)
  double* part;       // partial buffer for dense A^T (chunks x n)
  int chunks;         // row chunks of the dense A^T product
};

// Preconditioner P^{-1} z = z + V (d .* (V^T z)), V = Q_R V_M (n x ell).
// Explicit form (dense A): V row-major n x ell.  Implicit form (CSR A): with
// R = A(I,:) and Q_R = R^T T_R^{-1}, V = R^T K, K = T_R^{-1} V_M; the
// coefficients are c1 = R z, c2 = d .* (K^T c1), c = K c2 (or c = M2 c1 with
// M2 = K diag(d) K^T, one product instead of two, when R is well conditioned)
// and the row pass adds R^T c (CSR of R^T).
struct PrecDesc {
  int implicit;
  int ell;
  const double* d;
  double* c;      // ell
  // explicit: P^{-1} z = z + V (d .* (V^T z)), or z + V (M2 (V^T z)) when M2 is set
  long long ldv;
  const double* V;
  double* part;   // chunks x ell
  int chunks;
  // implicit: P^{-1} z = z + R^T (M (R z)), M = K diag(d) K^T as Kr (d .* (Kt .)) or M2
  const int* I;                    // rows of A forming R
  const double *Kt, *Kr;           // K^T and K, row-major ell x ell
  const double* M2;                // the middle ell x ell matrix (row-major) when used instead of Kt / Kr /
                                   // d, else null
  const double* M2t;               // M2^T (row-major) for the transpose apply P^{-T} when M2 is not
                                   // symmetric (the SVD-free form), else null
  const int *rt_ptr, *rt_idx;      // CSR of R^T (n rows)
  const double* rt_val;
  double *c1, *c2;                 // ell
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

// st points to the two state slots: slot 0 is written by the kernel that
// finishes alpha (scalar step), slot 1 by the kernel that finishes beta.
template <class V>
void gk_iteration(const OpDesc& A, const PrecDesc* P, GKVecs<V> vec, GKState* st, GKWork& wk, hipStream_t s);
// Phase start: r = [b - A x; bot_scale b_bot - delta x] computed in FP64 with
// Ares (b or b_bot may be null = 0; x null = 0) and stored in vec.u (type V),
// beta_1 = ||r||, v_1 = P^{-T} A_mu^T u_1 with A (alpha finished by the first
// kernel of the first iteration).  Ares and A describe the same matrix; A
// may hold FP32 values for the low-precision phases.
template <class V>
void gk_phase_init(const OpDesc& Ares, const OpDesc& A, const PrecDesc* P, const double* b, const double* b_bot,
                   double bot_scale, const double* x, GKVecs<V> vec, GKState* st, GKWork& wk, hipStream_t s);
// Phase end: x += P^{-1} y.
template <class V>
void gk_phase_finish(const OpDesc& A, const PrecDesc* P, GKVecs<V> vec, double* x, GKState* st, hipStream_t s);
// ||A_mu^T r||^2 -> st[0].h2 for r = [b - A x; bot_scale b_bot - delta x].
// y = P^{-1} z (trans = false) or P^{-T} z (trans = true), FP64 (n entries).
void gk_precond_apply(const OpDesc& A, const PrecDesc& P, bool trans, const double* z, double* y, hipStream_t s);
void gk_normal_residual(const OpDesc& A, const double* b, const double* b_bot, double bot_scale, const double* x,
                        GKVecs<double> vec, GKState* st, GKWork& wk, hipStream_t s);
void gk_normal_vector(const OpDesc& A, const double* b, const double* b_bot, double bot_scale, const double* x,
                      double* r_top, double* r_bot, double* g, GKState* st, GKWork& wk, hipStream_t s);
void set_state(GKState* st, const GKState& h, hipStream_t s);
void op_atb_norm2(const OpDesc& A, const double* b, double* tmp_n, GKState* st, GKWork& wk, hipStream_t s);
void op_norm(const OpDesc& A, const double* b, const double* b_bot, double bot_scale, double* tmp_m, double* tmp_n,
             GKState* st, GKWork& wk, hipStream_t s);
void op_matvec(const OpDesc& A, int trans, const double* x, double* y, GKState* st, GKWork& wk, hipStream_t s,
               hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
template <class V>
void fill_zero(V* p, long long n, hipStream_t s);
// CSR-stream products: non-zeros per workgroup for a matrix, workgroups, and
// the ints of a row-block array ({first row, its first non-zero} per
// workgroup, plus the end).
int stream_t(long long nnz);
int lx_stream_t(long long nnz);  // non-zeros per row block of the LDS-resident A x kernel
// LDS-resident A x: used for CSR with at least kLxMinNnz non-zeros when n
// vector entries fit kLxMaxBytes of dynamic LDS (below that size, loading x
// into every workgroup's LDS costs more than the gathers it saves).
constexpr long long kLxMaxBytes = 160 * 1024 - 1024;
constexpr long long kLxMinNnz = 1500000;
// SELL-64 launch shape: slices per workgroup and workgroups.
void sell_layout(long long nslices, long long n, int* spw, int* grid);
void gk_prepare();               // once per process: kernel attributes
// A read and a write of every byte of buf (bytes a multiple of 16), enqueued
// on s: evicts other data from the caches (cold-cache timing).
void touch_buffer(void* buf, long long bytes, hipStream_t s);
// SELL-64 copy: slice widths (returns padded entries), then the fill.
long long sell_widths(const int* rp, long long m, int* wid_dev, std::vector<int>& wid_host, hipStream_t s);
template <class TA>
void sell_fill(const int* rp, const int* ci, const TA* val, long long m, const int* off_dev, const int* wid_dev,
               int* sci, TA* sval, hipStream_t s);
int stream_blocks(long long nnz, int T);
long long row_block_words(long long nnz, int T);
void build_row_blocks(const int* rp, long long m, long long nnz, int T, int* rb, hipStream_t s);

}  // namespace aplicur
