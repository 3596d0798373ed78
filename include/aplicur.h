/*
 * aplicur.h -- C ABI of the MI355X (gfx950) APLICUR library, libaplicur.so.
 *
 * APLICUR (Huh, Cartis, Nakatsukasa, "Adaptive LSQR Preconditioning from One
 * Small Sketch") solves the regularised linear least-squares problem of
 * Sec. 1 (eq. (1.1)),
 *
 *        min_x ||A x - b||_2^2 + mu ||x||_2^2 ,    A in R^{m x n}, mu >= 0,
 *
 * by LSQR on the augmented operator A_mu = [A; sqrt(mu) I] (Sec. 2.1), right-
 * preconditioned by a CUR-based spectral preconditioner (Sec. 3.1, Alg. 2)
 * whose rank grows adaptively from one small sparse sign sketch S A
 * (Definition 5.1, Alg. 7) and which is rebuilt only when the CUR error
 * estimate has improved enough (Sec. 5.3, Alg. 3).
 *
 * Conventions common to every entry point
 *  - Every pointer argument is a DEVICE pointer unless marked (host).
 *  - The caller owns every buffer it passes; the library never frees them.
 *    The opaque context owns the device memory the library allocates itself
 *    (sketch, CUR factors, preconditioner, work vectors) and releases it in
 *    aplicur_ctx_destroy.
 *  - A is borrowed by the context: it must stay alive and unmodified until
 *    aplicur_ctx_destroy.
 *  - Right-hand sides B and solutions X are FP64, column-major (each column
 *    one right-hand side, contiguous), leading dimensions ldb >= m, ldx >= n.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream).
 *    The solve reads a few scalars back per outer step and per block of LSQR
 *    iterations, so the calls return only when their results are ready.
 *  - Return value: APLICUR_OK (0), a positive warning (results valid) or a
 *    negative error (outputs undefined).  aplicur_last_error() returns a
 *    thread-local message describing the last error of the calling thread.
 *  - Not thread-safe per context: one context must not be used from two
 *    threads at once.  Distinct contexts are independent.
 */
#ifndef APLICUR_H
#define APLICUR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
#define APLICUR_OK 0
#define APLICUR_W_MAXITER 1      /* iteration budget reached before tol_ne (x valid) */
#define APLICUR_E_INVALID (-1)   /* bad argument (shape, null pointer, option range) */
#define APLICUR_E_HIP (-3)       /* HIP runtime / rocBLAS failure */
#define APLICUR_E_BREAKDOWN (-4) /* non-finite value met (NaN/Inf in A or B, or overflow), or the
                                    first CUR block is singular; a later block whose columns are
                                    numerically dependent on C is dropped instead and ends the
                                    rank growth (Alg. 2, chol(C^T C)) */
#define APLICUR_E_NOMEM (-5)     /* device allocation failed */

/* ------------------------------------------------------------------ matrix */
#define APLICUR_DENSE 0 /* row-major m x n, leading dimension ld >= n            */
#define APLICUR_DENSE_COL 1 /* column-major m x n, leading dimension ld >= m: the
                               context keeps a row-major copy (m n values)        */
#define APLICUR_CSR 2   /* CSR: row_ptr[m+1], col_idx[nnz] (int32, any order), val[nnz] */
#define APLICUR_F64 0
#define APLICUR_F32 1

typedef struct aplicur_mat {
  int32_t format;         /* APLICUR_DENSE or APLICUR_CSR                     */
  int32_t dtype;          /* APLICUR_F64 or APLICUR_F32 (values of A)         */
  int64_t m, n;           /* rows, columns (m >= 1, n >= 1)                   */
  int64_t ld;             /* dense: leading dimension (elements), >= n        */
  int64_t nnz;            /* CSR: number of stored entries (< 2^31)           */
  const void* val;        /* dense: m*ld values; CSR: nnz values              */
  const int32_t* row_ptr; /* CSR only (device), else NULL                     */
  const int32_t* col_idx; /* CSR only (device), else NULL; no duplicates      */
} aplicur_mat;

/* ------------------------------------------------------------------ options
 * Hyper-parameters of Alg. 3 (defaults of Sec. 7 / App. C); fill with
 * aplicur_opts_default() and override.  Readings of the paper used here:
 * the objective weight mu enters A_mu as delta = sqrt(mu); the sketch has
 * s = ceil(1.1 block) rows (capped at m) with xi = min(8, s) non-zeros per
 * column; eps_cur <= 0 selects 30 sqrt(mu) (3e-7 when mu = 0).            */
typedef struct aplicur_opts {
  int32_t block;     /* rank increment b of Alg. 3 (1..280); sketch dim s = ceil(1.1 b)  */
  int32_t r_probes;  /* Gaussian probes of the 2-norm bound (Sec. 5.3.1), 1..64, default 10 */
  uint64_t seed;     /* seed of the sketch / probe stream (SplitMix64)                     */
  double mu;         /* regularisation weight, >= 0                                        */
  double eps_cur;    /* CUR tolerance on rho; <= 0: default reading                        */
  double nu_prec;    /* re-preconditioning tolerance (default 10)                          */
  double nu_lsqr;    /* dynamic LSQR stopping tolerance (default 100)                      */
  double eps_lsqr;   /* Paige-Saunders tolerance of intermediate phases (default 1e-10)    */
  double tol_ne;     /* requested ||A^T(b-Ax) - mu x|| / ||A^T b|| (default 1e-8)         */
  int32_t max_iter;  /* LSQR iteration budget per right-hand side (default 100000)         */
  int32_t max_rank;  /* cap on the CUR rank l (<= 0: min(m, n, 4096)); reaching it ends the
                        rank growth like rho <= eps_cur                                      */
  int32_t precond;   /* 1: APLICUR (default); 0: plain LSQR on A_mu (no sketch, no CUR);
                        2: APLICUR with the SVD-free preconditioner (Alg. 8, Sec. 3.1):
                        P~^{-1} = t Q_R M^{-1} Q_R^T + (I - Q_R Q_R^T), M^{-1} =
                        T_R^{-T} A(I,J) T_C^{-1}, target level t = max(rho, eps_cur);
                        applied through the orthonormal Q_R (n x l, dense and CSR A);
                        mu = 0 only
                        (E_INVALID otherwise); one right-hand side at a time        */
  int32_t precision; /* 0: FP64 vectors and products (default); 1: FP32 LSQR phases (FP32
                        values and vectors, FP64 scalars and reductions) with FP64
                        refinement (an extension, not in the paper); 2: as 1, and where
                        the columns run blocked (dense A, nrhs >= 2) the products of the
                        FP32 phases read BF16 copies of A and A^T (16x16x32 BF16 MFMA,
                        FP32 accumulation, the FP32 input split into two BF16 parts); a
                        BF16 phase stops at 1e-2 of its starting residual, and once a
                        BF16 phase divides some column's eta by less than 10 the rest of
                        that solve uses the FP32 products.  The copies (2 bytes per entry
                        each, tiles of 32 x 64) are made on first use and held until the
                        context is destroyed.  One column at a time, 2 behaves as 1      */
  int32_t max_outer; /* stop after this many outer steps (<= 0: no limit; for tests)       */
  int32_t workers;   /* aplicur_solve_batched: problems in flight at once, each on a stream
                        of its own (<= 0: 4)                                                  */
  int32_t tune;      /* 1: time candidate workgroup tiles of the product kernels on this
                        matrix at set-up and keep the fastest (cached per shape); 0: fixed
                        heuristic tiles.  Tiles change the summation order, not the method */
  int32_t graphs;    /* 1: replay the LSQR iterations as captured HIP graphs (same kernels,
                        same arithmetic); 0: launch each kernel                             */
  int32_t columns;   /* 1: one right-hand side at a time even where the blocked path applies
                        (several right-hand sides of a dense A); 0: blocked there
                        (default).  Same method and stopping tests per column              */
  int32_t xi;        /* non-zeros per column of the sparse sign sketch, 1..8 (default 8,
                        Sec. 5.1; 0 selects the default); the sketch uses min(xi, s)     */
  int32_t sketch;    /* 0: sparse sign embedding (default); 1: Gaussian embedding, i.i.d.
                        N(0, 1/s) entries from the counter-based stream 3 (Sec. 5.1), Y = S A by
                        the library's MFMA products: FP64 GEMM for FP64 A; for FP32 A, S
                        rounded to FP32, FP32 MFMA sums of 16 terms accumulated in FP64; a
                        column-wise kernel over the CSR of A^T for CSR A; 2: as 1, but for
                        dense FP32 A both S and A rounded to BF16 (BF16 MFMA, 32-term FP32
                        sums accumulated in FP64; about 2^-8 relative to |S| |A| per entry) */
  int32_t schedule;  /* 0: fully adaptive (default, Alg. 3: phases interleaved with the rank
                        growth and the re-preconditioning test); 1: rank-adaptive single
                        shot (the rank grows until rho <= eps_cur or the cap, then one P and
                        one final phase); 2: fixed-rank single shot (the rank grows to the
                        cap max_rank, then one P and one final phase).  Sec. 7.1       */
  double jacobi_tol; /* accuracy of the SVD of the l x l core M (Alg. 2 Part 2), by one-sided
                        Jacobi: sweeps stop once the Frobenius norm of the off-diagonal of
                        the damped core's Gram matrix, scaled to unit diagonal, is at most
                        this (as summed over the last sweep, or measured on the state a
                        sweep left); the preconditioned singular values then lie within
                        sqrt(1 +- jacobi_tol) of the exact-SVD level.  <= 0: 1e-2
                        (default); tiny values run the sweeps to convergence (at most 40) */
  int32_t tc_sketched; /* T_C (Alg. 2) when the Cholesky of C^T C breaks down after a CUR
                        increment (the new columns nearly dependent on C): 0 (default): the
                        increment is undone and the rank growth ends; 1: T_C is recomputed by
                        sketched Cholesky QR of C (Gaussian embedding of 2 l rows from stream 3
                        of seed + 7919, two shifted and two plain Cholesky QR passes on the
                        sketch, then one Cholesky QR of C R^{-1}), the growth continues, and
                        the increment is undone only if that breaks down too          */
} aplicur_opts;

/* ------------------------------------------------------------------ info  */
typedef struct aplicur_info { /* (host) */
  int32_t status;      /* same value as returned                                  */
  int32_t phases;      /* LSQR phases run (max over right-hand sides)             */
  int32_t iters;       /* LSQR iterations (max over right-hand sides)             */
  int32_t rank;        /* final CUR rank l                                         */
  int32_t rebuilds;    /* preconditioner builds                                    */
  int32_t outer;       /* outer (rank-increment) steps                             */
  int32_t phases_bf16; /* phases of the blocked path whose products read the BF16
                          copies of A (precision 2; 0 otherwise)                   */
  int32_t reserved;
  double eta;          /* max over columns of the final eta, FP64 from a fresh residual */
  double rho;          /* last CUR error estimate                                  */
  double sigma_hat;    /* last target level sqrt(sigma_l^2 + mu)                   */
  double t_sketch_ms, t_cur_ms, t_precond_ms, t_lsqr_ms; /* time split (host clock) */
} aplicur_info;

typedef struct aplicur_ctx aplicur_ctx;

/* Default options (Alg. 3 defaults: block 20, nu_prec 10, nu_lsqr 100,
 * eps_lsqr 1e-10, tol_ne 1e-8, r_probes 10, seed 7, mu 0).                */
void aplicur_opts_default(aplicur_opts* opts /* (host) */);

/* Device memory a context needs for solves (and adjoint solves) with up to
 * nrhs right-hand sides: its set-up buffers (sketch, CUR and preconditioner
 * storage sized by the rank cap, product layouts, LSQR vectors), the blocked
 * path's buffers for that many columns of a dense A (and the BF16 copies at
 * precision 2), and the transient blocks of the set-up and of the adjoint.
 * It is measured, not estimated: the call runs the set-up of A once on
 * `stream` with library-allocated memory and releases it.  A context used
 * with more columns than sized for runs out of its workspace (E_NOMEM).
 * Returns the byte count (> 0) or a negative error (E_INVALID, E_NOMEM,
 * E_HIP).  A, opts: (host).                                                */
int64_t aplicur_workspace_bytes(const aplicur_mat* A, int32_t nrhs, const aplicur_opts* opts, void* stream);

/* Set-up of Alg. 3 (initialisation): validates A, builds the CSR of A^T
 * (CSR input), draws the sparse sign embedding S (s x m) and the probes, and
 * forms the sketch Y = S A in FP64 once (Alg. 3, initialisation; Sec. 5.1).
 * A (host struct) describes device arrays, borrowed until ctx destruction.
 * opts (host) is copied.  *ctx_out (host) receives the new context.
 * ws (device, optional): a caller workspace of ws_bytes bytes, 256-byte
 * aligned, owned by the caller and untouched after ctx destruction; every
 * device buffer of the context is carved from it (size it with
 * aplicur_workspace_bytes).  ws = NULL: the library allocates with
 * hipMalloc and frees at destruction.  Either way small pinned host buffers
 * hold the read-backs.  Errors: E_INVALID (shape/options/alignment), E_NOMEM
 * (allocation failed or workspace exhausted), E_HIP.                       */
int aplicur_sketch(const aplicur_mat* A, const aplicur_opts* opts, void* ws, size_t ws_bytes, void* stream,
                   aplicur_ctx** ctx_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the sketch
 * Y = S A of aplicur_sketch (Alg. 3 initialisation, the sparse sign embedding
 * of Definition 5.1 with the same seed, block and xi options, so the same S)
 * written into caller memory, with no context and no device allocation.
 * Y (device): s x n doubles, row-major, s = min(m, ceil(1.1 block)).  A as in
 * aplicur_sketch, but row-major dense or CSR (APLICUR_DENSE_COL: E_INVALID);
 * opts.precond must be 1 or 2 and opts.sketch 0.  Scratch (the sketch's rows
 * and signs; for CSR A the validation flag and the CSR of A^T; for dense A the
 * inverse of the embedding, 4 xi m bytes and a few per target row) lives in
 * a fixed array of 64 MiB per device that the library holds until the
 * process ends; an input whose scratch would exceed it is rejected
 * (E_INVALID, the message gives the bytes needed) before any device work.
 * The result equals aplicur_sketch's bit for bit (same kernels, same
 * summation order).  Calls on one device share that array: calls that overlap on
 * one GPU (different streams, or different host threads) race; serialise
 * them.  CSR validation reads one flag back (the call synchronises the
 * stream).  Errors: E_INVALID, E_HIP.                                       */
int aplicur_sketch_noalloc(const aplicur_mat* A, const aplicur_opts* opts, double* Y, void* stream);

/* The adaptive solve of Alg. 3 for nrhs right-hand sides B (m x nrhs,
 * column-major, ldb >= m) into X (n x nrhs, ldx >= n).  All columns share
 * the CUR sequence and every preconditioner (none depends on b); each
 * column runs its own LSQR recurrences with its own dynamic stopping.  For
 * a dense A with nrhs >= 2 (any precision) the columns run together, up to
 * 64 at a time, sharing each product (one pass over A per iteration for
 * the group; A^T products read a transposed copy of A made on first use,
 * held until the context is destroyed); otherwise one column at a time.  With
 * x_is_warm != 0 the first phase starts from the given X (warm start,
 * Sec. 3.2), otherwise from 0.  The context remembers the final CUR state
 * and preconditioner for aplicur_solve_backward.  info (host) may be NULL.
 * Returns OK, W_MAXITER, or an error.                                      */
int aplicur_solve(aplicur_ctx* ctx, const double* B, int64_t ldb, int32_t nrhs, double* X, int64_t ldx,
                  int32_t x_is_warm, aplicur_info* info, void* stream);

/* Independent problems A[p] x = B[p] (p < batch) with the same options
 * (batching is an extension, not in the paper): A, B, ldb, X, ldx and info
 * are (host) arrays of length batch; B[p] / X[p] are device pointers (FP64,
 * column-major, nrhs columns each).  opts.workers host threads each own a
 * HIP stream (default priority) that first waits for `stream`, and take
 * whole problems, largest first; each problem runs Alg. 3 through the same
 * kernels as aplicur_solve (opts.graphs: its LSQR iterations replay as HIP
 * graphs; opts.tune: product tiles autotuned per shape).  All work is done
 * when the call returns.  Every problem is validated before any work starts.
 * ws (device, optional): a caller workspace of ws_bytes bytes, 256-byte
 * aligned, sized with aplicur_batched_workspace_bytes: worker w carves the
 * context of every problem it runs from slice w (each slice fits the largest
 * problem's context), so the call allocates no device memory for contexts;
 * ws = NULL: each context allocates with hipMalloc and frees when its
 * problem is done.  Errors: E_INVALID (also a workspace below the size the
 * call needs; the message gives it), E_NOMEM, E_HIP.  Returns the first
 * error (naming the problem), else the largest warning.                     */
int aplicur_solve_batched(int32_t batch, const aplicur_mat* A, const double* const* B, const int64_t* ldb,
                          int32_t nrhs, double* const* X, const int64_t* ldx, const aplicur_opts* opts,
                          void* ws, size_t ws_bytes, aplicur_info* info, void* stream);

/* Workspace bytes of aplicur_solve_batched for these problems, nrhs and
 * options: min(batch, opts.workers (0: 4)) slices, each the largest context
 * any problem needs (measured as aplicur_workspace_bytes does, by running
 * each problem's set-up once on `stream` with library-allocated memory).
 * Returns the byte count (> 0) or a negative error (E_INVALID, E_NOMEM,
 * E_HIP).                                                                    */
int64_t aplicur_batched_workspace_bytes(int32_t batch, const aplicur_mat* A, int32_t nrhs, const aplicur_opts* opts,
                                        void* stream);

/* Adjoint of the solve (not in the paper; implicit differentiation of the
 * normal equations A^T (B - A X) = mu X).  For a loss with G = dL/dX
 * (n x nrhs, ldg), computes
 *    Z  = (A^T A + mu I)^{-1} G     by preconditioned LSQR on A_mu with the
 *                                    right-hand side [0; G / sqrt(mu)] and
 *                                    the context's final preconditioner,
 *    dB = A Z                        (m x nrhs, lddb)          = dL/dB,
 *    dA = (B - A X) Z^T - (A Z) X^T  (dense A: m x n in A's layout,
 *                                    row-major with ldda >= n, or
 *                                    column-major with ldda >= m; CSR A:
 *                                    nnz values on the sparsity pattern) = dL/dA.
 * X, B are the forward solution and right-hand sides.  Requires mu > 0 and
 * a context on which aplicur_solve has run.  dA may be NULL (skipped); Z
 * (n x nrhs, ldz) receives Z.  Errors: E_INVALID, E_HIP, E_BREAKDOWN.      */
int aplicur_solve_backward(aplicur_ctx* ctx, const double* X, int64_t ldx, const double* B, int64_t ldb,
                           const double* G, int64_t ldg, int32_t nrhs, double* Z, int64_t ldz, double* dB,
                           int64_t lddb, double* dA, int64_t ldda, aplicur_info* info, void* stream);

/* y = A x (trans = 0; x: n, y: m) or y = A^T x (trans = 1; x: m, y: n) in
 * FP64 with the same product kernels the LSQR iteration uses.             */
int aplicur_matvec(aplicur_ctx* ctx, int32_t trans, const double* x, double* y, void* stream);

/* Y[:, j] = A X[:, j] (trans = 0) or A^T X[:, j] (trans = 1) for j < k: X and
 * Y device, FP64, column-major with leading dimensions ldx >= (trans ? m : n)
 * and ldy >= (trans ? n : m).  Dense A: one pass over A (or over its
 * transposed copy, made on first use) for up to 64 columns at a time on
 * MFMA (the products of the blocked multi-right-hand-side LSQR, Sec. 2.2);
 * prec selects the arithmetic of the products the phases use:
 *   0: FP64 accumulation of the stored FP32/FP64 values;
 *   1: X rounded to FP32, FP32 values, FP32 accumulation (the FP32 phases;
 *      a context of precision 1 or 2);
 *   2: the BF16 copies of A / A^T, X split into two BF16 parts, FP32
 *      accumulation (the BF16 products of precision 2).
 * CSR A: one FP64 product per column (prec 0 only).  Enqueued on `stream`.
 * Errors: E_INVALID (arguments, prec not available), E_HIP.               */
int aplicur_matmat(aplicur_ctx* ctx, int32_t trans, const double* X, int64_t ldx, int32_t k, double* Y, int64_t ldy,
                   int32_t prec, void* stream);

/* y = P^{-1} z (trans = 0) or y = P^{-T} z (trans = 1) with the context's
 * last preconditioner (Alg. 2 Part 2: P^{-1} z = z + V ((sigma/Lambda - 1) .*
 * (V^T z)), V = Q_R V_M, symmetric; or the SVD-free P~^{-1} of Alg. 8, whose
 * transpose differs), through the same kernels as the one-column LSQR
 * iteration (the implicit R^T K form for CSR A, the explicit V for dense A;
 * the first call after a solve with several right-hand sides, which applies
 * P as z + Q_R W Q_R^T z with W = V_M diag(sigma/Lambda - 1) V_M^T, forms V
 * once on `stream`).  z, y: n doubles (device), distinct.  Enqueued on
 * `stream`.  For tests and diagnostics.  Errors: E_INVALID (null argument,
 * no preconditioner built yet: run aplicur_solve first), E_HIP.           */
int aplicur_precond_apply(aplicur_ctx* ctx, int32_t trans, const double* z, double* y, void* stream);

/* Measures the product kernels the LSQR iteration uses: `reps` rounds of
 * y = A x - y followed by s = A^T y (s: library scratch), alternating as in
 * the iteration, with a HIP event pair attached to every dispatch of the A
 * product (trans = 0) or of the A^T product (trans = 1) on `stream`
 * (hipExtLaunchKernelGGL start/stop events).
 * x: n doubles, y: m doubles (scratch; final contents unspecified).
 * flush (device, optional): a caller buffer of flush_bytes bytes (a
 * multiple of 16; contents overwritten) that is read and written before
 * each round, so that the timed product finds its matrix in neither L2
 * nor the 256 MB last-level cache (cold-cache timing; give at least 512
 * MB).  NULL: warm caches, as in the LSQR loop.
 * *us_per_launch (host) receives the mean duration in microseconds.
 * Errors: E_INVALID, E_HIP.                                                */
int aplicur_time_product(aplicur_ctx* ctx, int32_t trans, const double* x, double* y, int32_t reps, void* flush,
                         int64_t flush_bytes, void* stream, double* us_per_launch);

/* Measures the blocked product kernel of the several-right-hand-side path
 * (dense A): `reps` calls of Y = A X (trans = 0) or A^T X (trans = 1) for k
 * columns (1 <= k <= 64) in the arithmetic prec of aplicur_matmat, with a
 * HIP event pair attached to the dispatch of the product kernel itself (the
 * MFMA row-streaming kernel that reads A once; the packing and partial-sum
 * kernels around it are not timed).  X, Y: column-major FP64 (device),
 * ldx >= (trans ? m : n), ldy >= (trans ? n : m).  flush: as in
 * aplicur_time_product (cold caches), or NULL.  One untimed call first makes
 * any copy of A the product needs.  *us_per_launch (host) receives the mean
 * kernel duration in microseconds.  Errors: E_INVALID, E_HIP.             */
int aplicur_time_matmat(aplicur_ctx* ctx, int32_t trans, const double* X, int64_t ldx, int32_t k, double* Y,
                        int64_t ldy, int32_t prec, int32_t reps, void* flush, int64_t flush_bytes, void* stream,
                        double* us_per_launch);

/* Event timing of the blocked product kernel inside solves (measurement of
 * the several-right-hand-side path of Sec. 2.2's products, dense A): while
 * enabled, every dispatch of the row-streaming product kernel, by any
 * context of this process on the device that was current at enable time,
 * carries a HIP event pair taking the kernel's own start and end (at most
 * 65536 launches between reads; later ones are counted as untimed).  The
 * events are created on first use and reused, so a warm-up with timing on
 * keeps event creation out of a later timed region.  enable = 0 stops
 * timing and keeps the record.  Switching device needs an empty record.
 * Errors: E_INVALID, E_HIP.                                                  */
int aplicur_prof_products(int32_t enable);

/* Reads and clears the record of aplicur_prof_products, waiting for the
 * recorded launches: per kind k (0: A X, 1: A^T X with FP64 accumulation;
 * 2, 3: the same with FP32 products; 4, 5: with BF16 products) the timed
 * launches, their summed kernel durations in microseconds, and the launches
 * left untimed.  All three arrays (host) hold 6 entries.
 * Errors: E_INVALID, E_HIP.                                                  */
int aplicur_prof_read(int64_t* launches, double* total_us, int64_t* untimed);

/* Read internal state back to host memory (tests and diagnostics).
 * what: 1 sketch Y (s x n row-major doubles), 2 sketch rows (m x xi int32;
 * none for the Gaussian sketch),
 * 3 sketch signs (m x xi int32, +-1), 4 probes (n x r doubles, column-major),
 * 5 column indices J (rank int32), 6 row indices I (rank int32),
 * 7 rho history (outer doubles), 8 rank history (outer int32),
 * 9 rebuild flags (outer int32), 10 sizes {m, n, s, xi, rank, outer, r} (int64),
 * 11 last preconditioner singular values sigma (rank doubles),
 * 12 per-phase iteration counts of column 0 (int32), 13 per-phase eta of column 0 (doubles),
 * 14 Jacobi sweeps of each preconditioner build (int32; 0 for the SVD-free form),
 * 15 the middle matrix H = t M^{-1} - I of the last SVD-free preconditioner
 * (P~^{-1} z = z + Q_R H Q_R^T z; rank x rank doubles, row-major; none
 * otherwise).
 * Returns the number of bytes available (copies min(bytes, available)), or
 * a negative error.                                                        */
int64_t aplicur_ctx_query(const aplicur_ctx* ctx, int32_t what, void* host_out, size_t bytes);

void aplicur_ctx_destroy(aplicur_ctx* ctx);
const char* aplicur_last_error(void);
const char* aplicur_version(void);

#ifdef __cplusplus
}
#endif

#endif /* APLICUR_H */
