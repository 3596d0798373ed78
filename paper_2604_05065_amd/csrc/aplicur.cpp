// Host driver of the APLICUR library: the adaptive procedure of Alg. 3 on
// the GPU, and the extern "C" entry points declared in include/aplicur.h.
//
// Per outer step (Alg. 3 Part 1-3):
//   augmentCUR (Alg. 7): zero E_row(:,J); LUPP pivots of E_row^T -> J+;
//     E_col = A(:,J+) - C (U R(:,J+)); zero E_col(I,:); LUPP pivots -> I+;
//   U = A(I,J)^{-1} kept explicitly and extended by the block-inverse formula
//     with the Schur complement S = E_col(I+, :) (the LU pivot block);
//   E_row = Y - (Y(:,J) U) R;  rho = 10 sqrt(2/pi) max_i ||E_row w_i||;
//   augmentQR (Alg. 9) of R^T (CGS2 + Cholesky QR of the remainder);
//   T_C = chol(C^T C) extended by the same block recurrence;
//   if re-preconditioning: M = T_C U T_R^T, one-sided Jacobi SVD of M,
//     V = Q_R V_M, P^{-1} z = z + V ((sigma^/Lam - 1) .* V^T z), then an LSQR
//     phase per right-hand side warm-started from x.
// The GEMM / TRSM steps run on the library's own FP64 MFMA kernels (kern_blas.hip).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <shared_mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/aplicur.h"
#include "blas.h"
#include "blk.h"
#include "factor.h"

namespace aplicur {

static thread_local std::string g_last_error;
void set_last_error(const std::string& msg) { g_last_error = msg; }

// Host calls that may synchronise with the legacy stream behind the scenes
// (allocation and release, library handles, library calls, which may load or
// set up kernels on first use) hold this lock shared; capturing a graph holds
// it exclusively, because such a call from another thread during a capture
// is an error.
static std::shared_mutex g_capture_mu;
using SyncGuard = std::shared_lock<std::shared_mutex>;

using Clock = std::chrono::steady_clock;
static double ms_since(Clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

// Device arena: every allocation of a context, released together.
// Device buffers of a context: from hipMalloc, or carved (256-byte aligned)
// from a caller workspace [base, base + cap).  used counts the aligned bytes
// of the permanent buffers, peak the most ever needed at once (permanent
// plus the largest transient one): the workspace a context needs.
struct Arena {
  std::vector<void*> ptrs;
  char* base = nullptr;
  size_t cap = 0, used = 0, peak = 0;
  static constexpr size_t kAlign = 256;
  static size_t aligned(size_t bytes) { return (std::max<size_t>(bytes, 1) + kAlign - 1) / kAlign * kAlign; }
  void room(size_t bytes) const {
    if (bytes > cap - used)
      throw Error(APLICUR_E_NOMEM, "workspace of " + std::to_string(cap) + " bytes exhausted (" +
                                       std::to_string(used) + " used, " + std::to_string(bytes) +
                                       " more requested); size it with aplicur_workspace_bytes");
  }
  // A transient buffer that lives until the next alloc: in workspace mode the
  // space after the permanent buffers (owned = false), else a hipMalloc the
  // caller frees (owned = true).
  void* transient(size_t bytes, bool& owned) {
    bytes = aligned(bytes);
    peak = std::max(peak, used + bytes);
    owned = base == nullptr;
    if (base) {
      room(bytes);
      return base + used;
    }
    void* p = nullptr;
    SyncGuard g(g_capture_mu);
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      throw Error(APLICUR_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    return p;
  }
  template <class T>
  T* alloc(size_t count) {
    if (count == 0) count = 1;
    const size_t bytes = aligned(count * sizeof(T));
    if (base) {
      room(bytes);
      void* p = base + used;
      used += bytes;
      peak = std::max(peak, used);
      return (T*)p;
    }
    used += bytes;
    peak = std::max(peak, used);
    void* p = nullptr;
    SyncGuard g(g_capture_mu);
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error(APLICUR_E_NOMEM, "device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed");
    }
    ptrs.push_back(p);
    return (T*)p;
  }
  void release() {
    SyncGuard g(g_capture_mu);
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
  }
};

constexpr int kLuppNB = 32;  // pivots per panel of the blocked LU pivot search
constexpr double kJacobiTol = 1e-2;  // default stopping level of the core SVD (see build_precond)

// Buffers of the blocked path (several right-hand sides of a dense A),
// allocated on first use for kp columns.
struct Blk {
  int kp = 0;
  void* At = nullptr;  // A^T, n x ldt row-major
  long long ldt = 0;
  double* W = nullptr;  // V_M diag(d) V_M^T of the explicit P, ell x ell (symmetric)
  long long w_gen = -1;
  double *Bp = nullptr, *Bbot = nullptr, *Xp = nullptr, *tm = nullptr, *tn = nullptr;
  BlkVecs<double> vec{};
  BlkWork wk{};
  BlkOp op{};
  // precision 1: the FP32 operator (FP32 values of A and of A^T), FP32 block
  // vectors, and the right-hand side of the refinement corrections
  BlkOp op32{};
  void* At32 = nullptr;
  BlkVecs<float> vec32{};
  double* Nc = nullptr;
  // precision 2: op32 with BF16 tiled copies of A and A^T for the products;
  // bf16_live is cleared for the rest of a solve once a BF16 phase gains too
  // little, last_bf16 says whether the last phase used them
  BlkOp op16{};
  void *A16 = nullptr, *At16 = nullptr;
  bool bf16_live = false, last_bf16 = false;
  int phases16 = 0;
  GKState* st = nullptr;
  GKState* st_up = nullptr;    // pinned, 2 kp (uploads)
  GKState* st_down = nullptr;  // pinned, 2 kp (read-backs)
  double* norm_host = nullptr; // pinned, kBlkMaxGrid x kp
  int S1max = 1, S2max = 1;
  // The last normal-residual evaluation (blk_col_norms, mode 1: A^T B; mode
  // 2: r = [B - A X; bs Bbot - delta X] in tm / tn and A^T r_top in wk.pn,
  // FP64).  The next FP64 phase start on the same B, bottom block and X takes
  // r_top and the planes from there instead of running both products again.
  // Cleared by every phase and by anything else that writes Bp, Xp, tm, tn or
  // wk.pn.
  struct {
    bool ok = false, x_zero = false;
    const double* Bbot = nullptr;
    double bs = 0.0;
  } nres;
};

struct Ctx {
  aplicur_mat A{};
  aplicur_opts o{};
  OpDesc op{};
  hipStream_t stream = nullptr;  // the stream of the current call (set_stream)
  double* nrm_tmp = nullptr;     // dnrm2 partials
  Arena arena;
  long long m = 0, n = 0;
  int s = 0, xi = 0, r = 0, L = 0, Lpad = 0, bmax = 0;
  double delta = 0.0, eps_cur = 0.0;
  double jacobi_tol = 0.0;  // stopping level of the core SVD's Jacobi sweeps
  // sketch / probes
  uint16_t* S_rows = nullptr;
  uint8_t* S_neg = nullptr;
  double *Y = nullptr, *E = nullptr, *W = nullptr, *EW = nullptr, *rho_dev = nullptr;
  // CUR state
  int *I_dev = nullptr, *J_dev = nullptr, *Ip = nullptr, *Jp = nullptr;
  std::vector<int> I, J;
  double *C = nullptr, *Rt = nullptr, *U = nullptr, *Q = nullptr, *TR = nullptr, *TC = nullptr;
  double *Ecol = nullptr, *RJ = nullptr, *F = nullptr, *Gm = nullptr, *H = nullptr, *Sb = nullptr,
         *Sinv = nullptr, *B21 = nullptr, *YJ = nullptr, *Z = nullptr, *P2 = nullptr, *small = nullptr;
  int* status_dev = nullptr;
  int* lu_piv = nullptr;  // pivots of the blocked LU of the Schur block
  int rank = 0;
  // preconditioner
  double *Mx = nullptr, *Vm = nullptr, *sigma = nullptr, *Vhat = nullptr, *d = nullptr, *pinfo = nullptr,
         *pa_part = nullptr, *pa_c = nullptr, *Kc = nullptr, *Kr = nullptr, *pc1 = nullptr, *pc2 = nullptr,
         *M2 = nullptr, *M2t = nullptr;
  int *rr_ptr = nullptr, *rr_idx = nullptr, *rt_ptr = nullptr, *rt_idx = nullptr, *rscratch = nullptr;
  double *rr_val = nullptr, *rt_val = nullptr;
  double* jac_part = nullptr;  // Jacobi scratch: stopping partials, pair Grams and rotations
  double* splitk = nullptr;
  size_t splitk_count = 0;
  PrecDesc prec{};
  bool have_prec = false;
  // what Vhat holds for the explicit P of generation vhat_gen: 1 V = Q_R V_M
  // (one-column paths), 2 Q_R row-major (blocked path), 0 nothing yet
  int vhat_kind = 0;
  long long vhat_gen = -1;
  int vm_rank = 0;       // rank of the right singular vectors held in Vm (warm start of the next build)
  long long vm_ld = 0;   // their leading dimension
  double p_target = 0.0, p_pnorm = 1.0, p_sigma_l = 0.0;
  std::vector<double> p_sigma_host;
  // LSQR vectors and state (FP64; FP32 copies for the low-precision phases)
  double *u_top = nullptr, *u_bot = nullptr, *v = nullptr, *w = nullptr, *y = nullptr, *t = nullptr,
         *g = nullptr;
  bool fp32 = false;
  bool bf16 = false;  // precision 2: BF16 copies for the blocked products of the FP32 phases
  OpDesc op32{};  // the same matrix with FP32 values (precision 1)
  float *u_top32 = nullptr, *u_bot32 = nullptr, *v32 = nullptr, *w32 = nullptr, *y32 = nullptr, *t32 = nullptr,
        *g32 = nullptr;
  GKWork wk{};
  GKState* st = nullptr;       // two state slots
  GKState* st_host = nullptr;  // pinned, two slots
  GKState* st_mv = nullptr;    // two slots of the matvec entry point (alpha = beta = 1, delta = 0)
  unsigned* counter = nullptr;
  FactorWork fw{};
  // histories
  std::vector<double> rho_hist;
  std::vector<int> rank_hist, rebuild_hist, sweep_hist;
  std::vector<int> phase_iters0;
  std::vector<double> phase_eta0;
  double t_sketch = 0.0;
  // captured LSQR iteration chunk (graphs option) and the key it was captured for
  hipGraphExec_t gexec = nullptr;
  long long gkey = -1;
  // blocked path and the generation of the preconditioner it last saw
  std::unique_ptr<Blk> blk;
  long long prec_gen = 0;

  ~Ctx() {
    {
      SyncGuard g(g_capture_mu);
      if (gexec) (void)hipGraphExecDestroy(gexec);
      if (st_host) (void)hipHostFree(st_host);
      if (blk) {
        if (blk->st_up) (void)hipHostFree(blk->st_up);
        if (blk->st_down) (void)hipHostFree(blk->st_down);
        if (blk->norm_host) (void)hipHostFree(blk->norm_host);
      }
    }
    arena.release();
  }
};

static int group_for(double avg) {
  int g = 1;
  while (g < avg && g < 64) g <<= 1;
  return g;
}

static void set_stream(Ctx& c, hipStream_t s) { c.stream = s; }

// Scratch of the k-chunked products (dgemm sums the chunk products in
// order): one fixed block per context, reserved at set-up, so that every
// product is cut the same way in every call and in both memory modes.
constexpr size_t kGemmWorkMax = size_t(4) << 20;  // doubles (32 MiB)

// C = alpha op(A) op(B) + beta C on the library's FP64 MFMA GEMM, on the
// context's current stream.
static void gemm(Ctx& c, Op ta, Op tb, long long m, long long n, long long k, double alpha, const double* A,
                 long long lda, const double* B, long long ldb, double beta, double* Cm, long long ldc) {
  if (m <= 0 || n <= 0) return;
  dgemm(ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, Cm, ldc, c.splitk, c.splitk_count, c.stream);
}

// B <- alpha op(T)^{-1} B or alpha B op(T)^{-1}.
static void trsm(Ctx& c, Side side, Uplo uplo, Op trans, Diag diag, long long m, long long n, double alpha,
                 const double* T, long long ldt, double* B, long long ldb) {
  dtrsm(side, uplo, trans, diag, m, n, alpha, T, ldt, B, ldb, c.splitk, c.splitk_count, c.stream);
}

static int read_int(const int* dev, hipStream_t s) {
  int h = 0;
  APL_HIP(hipMemcpyAsync(&h, dev, sizeof(int), hipMemcpyDeviceToHost, s));
  APL_HIP(hipStreamSynchronize(s));
  return h;
}

// ------------------------------------------------------------------ set-up
void validate(const aplicur_mat* A, const aplicur_opts* o) {
  APL_REQUIRE(A && o, "null matrix or options");
  APL_REQUIRE(A->m >= 1 && A->n >= 1, "m and n must be >= 1");
  APL_REQUIRE(A->m < (1LL << 31) && A->n < (1LL << 31), "m and n must be < 2^31");
  APL_REQUIRE(A->dtype == APLICUR_F64 || A->dtype == APLICUR_F32, "dtype must be F64 or F32");
  APL_REQUIRE(A->val != nullptr, "A.val is null");
  if (A->format == APLICUR_CSR) {
    APL_REQUIRE(A->row_ptr && A->col_idx, "CSR needs row_ptr and col_idx");
    APL_REQUIRE(A->nnz >= 0 && A->nnz < (1LL << 31), "nnz out of range");
  } else {
    APL_REQUIRE(A->format == APLICUR_DENSE || A->format == APLICUR_DENSE_COL, "format must be DENSE, DENSE_COL or CSR");
    APL_REQUIRE(A->ld >= (A->format == APLICUR_DENSE ? A->n : A->m),
                A->format == APLICUR_DENSE ? "dense ld must be >= n" : "column-major ld must be >= m");
  }
  APL_REQUIRE(o->mu >= 0.0 && std::isfinite(o->mu), "mu must be finite and >= 0");
  APL_REQUIRE(o->mu > 0.0 || A->m >= A->n, "mu = 0 needs m >= n");
  APL_REQUIRE(o->precision >= 0 && o->precision <= 2,
              "precision must be 0 (FP64), 1 (FP32 phases, FP64 refinement) or 2 (1 with BF16 blocked products)");
  APL_REQUIRE(o->precond >= 0 && o->precond <= 2, "precond must be 0 (plain LSQR), 1 (APLICUR) or 2 (SVD-free)");
  APL_REQUIRE(o->precond != 2 || o->mu == 0.0, "the SVD-free preconditioner (precond = 2) needs mu = 0");
  if (o->precond) {
    APL_REQUIRE(o->block >= 1 && o->block <= 280, "block must be in [1, 280]");
    APL_REQUIRE(o->r_probes >= 1 && o->r_probes <= 64, "r_probes must be in [1, 64]");
  }
  APL_REQUIRE(o->max_iter >= 0, "max_iter must be >= 0");
  APL_REQUIRE(o->xi >= 0 && o->xi <= 8, "xi must be in [1, 8] (0: the default 8)");
  APL_REQUIRE(o->sketch >= 0 && o->sketch <= 2,
              "sketch must be 0 (sparse sign), 1 (Gaussian) or 2 (Gaussian, BF16 products for FP32 A)");
  APL_REQUIRE(o->schedule >= 0 && o->schedule <= 2, "schedule must be 0, 1 or 2");
  APL_REQUIRE(std::isfinite(o->jacobi_tol) && o->jacobi_tol < 1.0, "jacobi_tol must be finite and < 1");
  APL_REQUIRE(o->tc_sketched == 0 || o->tc_sketched == 1, "tc_sketched must be 0 or 1");
}

// ------------------------------------------------------------------ product tiles
// Row chunks of the dense A^T product (partial column sums over m / chunks
// rows each, then an ordered sum): about 2048 workgroups in all.
static int dense_chunks(long long m, long long n) {
  long long chunks = (2048 + (n + 255) / 256 - 1) / ((n + 255) / 256);
  chunks = std::min<long long>(chunks, std::max<long long>(1, m / 32));
  return (int)std::max<long long>(1, std::min<long long>(chunks, 1024));
}

// Candidate non-zeros per CSR-stream workgroup (LDS holds 2048 products).
static constexpr int kTileT[3] = {1024, 1280, 1536};

// Mean of the fastest launches of the A product plus the A^T product, in
// microseconds, with A and A^T alternating as in the iteration (dispatch-timed events).
static double time_pair(Ctx& c, int reps, hipStream_t s) {
  std::vector<hipEvent_t> ev(4);
  {
    SyncGuard g(g_capture_mu);
    for (auto& e : ev) APL_HIP(hipEventCreate(&e));
  }
  double best_a = 1e30, best_t = 1e30;
  for (int i = 0; i < reps; ++i) {
    op_matvec(c.op, 0, c.v, c.u_top, c.st_mv, c.wk, s, ev[0], ev[1]);
    op_matvec(c.op, 1, c.u_top, c.g, c.st_mv, c.wk, s, ev[2], ev[3]);
    APL_HIP(hipEventSynchronize(ev[3]));
    float a = 0.f, t = 0.f;
    APL_HIP(hipEventElapsedTime(&a, ev[0], ev[1]));
    APL_HIP(hipEventElapsedTime(&t, ev[2], ev[3]));
    if (i > 0) {  // the first round warms the caches
      best_a = std::min(best_a, (double)a);
      best_t = std::min(best_t, (double)t);
    }
  }
  SyncGuard g(g_capture_mu);
  for (auto& e : ev) (void)hipEventDestroy(e);
  return 1e3 * (best_a + best_t);
}

static std::mutex g_tile_mu;
static std::map<std::tuple<int, int, long long, long long, long long>, int> g_tile_cache;

// Autotuner: times each candidate tile of the product kernels on this matrix
// (CSR: non-zeros per workgroup; dense: row chunks of A^T) and keeps the
// fastest; the choice is cached per shape for the process.
static void tune_tiles(Ctx& c, hipStream_t s) {
  OpDesc& op = c.op;
  const auto key = std::make_tuple(op.csr, op.f64, op.m, op.n, op.csr ? op.nnz : op.ld);
  int choice = -1;
  {
    std::lock_guard<std::mutex> lk(g_tile_mu);
    auto it = g_tile_cache.find(key);
    if (it != g_tile_cache.end()) choice = it->second;
  }
  std::vector<int> cand;
  if (op.csr)
    cand.assign(std::begin(kTileT), std::end(kTileT));
  else
    for (int f : {1, 2, 4})
      for (int d : {1, 2})
        if (f == 1 || d == 1) cand.push_back(std::max(1, std::min(1024, op.chunks * f / d)));
  auto apply = [&](int v) {
    if (op.csr) {
      op.stream_t = v;
      build_row_blocks(op.row_ptr, op.m, op.nnz, v, (int*)op.rb, s);
      build_row_blocks(op.t_ptr, op.n, op.nnz, v, (int*)op.t_rb, s);
    } else {
      op.chunks = v;
    }
  };
  if (choice < 0) {
    fill(c.v, c.n, 1.0, s);
    fill(c.u_top, c.m, 0.0, s);
    double best = 1e30;
    for (int v : cand) {
      apply(v);
      const double us = time_pair(c, 6, s);
      if (us < best) {
        best = us;
        choice = v;
      }
    }
    std::lock_guard<std::mutex> lk(g_tile_mu);
    g_tile_cache[key] = choice;
  }
  apply(choice);
  if (c.fp32) {
    c.op32.stream_t = op.stream_t;
    c.op32.chunks = op.chunks;
  }
  APL_HIP(hipStreamSynchronize(s));
}

static Ctx* create(const aplicur_mat* Am, const aplicur_opts* o, hipStream_t s, void* ws = nullptr,
                   size_t ws_bytes = 0) {
  validate(Am, o);
  {
    SyncGuard g(g_capture_mu);
    gk_prepare();
  }
  auto t0 = Clock::now();
  Ctx* c = new Ctx();
  c->arena.base = (char*)ws;
  c->arena.cap = ws ? ws_bytes : 0;
  try {
    c->A = *Am;
    c->o = *o;
    c->m = Am->m;
    c->n = Am->n;
    c->delta = std::sqrt(o->mu);
    c->eps_cur = o->eps_cur > 0 ? o->eps_cur : (o->mu > 0 ? 30.0 * std::sqrt(o->mu) : 3e-7);
    c->jacobi_tol = o->jacobi_tol > 0 ? o->jacobi_tol : kJacobiTol;
    set_stream(*c, s);
    c->nrm_tmp = c->arena.alloc<double>(kNrm2Parts + 1);
    {
      // k-chunk scratch of the set-up products: the tall products have at
      // most 64 chunks of (rank cap) x (block) or s x r outputs
      const long long L = std::min<long long>(std::min(Am->m, Am->n), o->max_rank > 0 ? o->max_rank : 4096);
      const long long b = std::max<long long>(1, std::min<long long>(o->block, 280));
      const size_t want = (size_t)64 * (size_t)(L * b + 2 * b * b + 310 * 64);
      c->splitk_count = std::min(kGemmWorkMax, want);
      c->splitk = c->arena.alloc<double>(c->splitk_count);
    }
    const long long m = c->m, n = c->n;
    OpDesc& op = c->op;
    op.csr = (Am->format == APLICUR_CSR);
    op.f64 = (Am->dtype == APLICUR_F64);
    op.m = m;
    op.n = n;
    op.ld = op.csr ? 0 : Am->ld;
    op.val = Am->val;
    if (Am->format == APLICUR_DENSE_COL) {
      // row-major copy: the column-major m x n matrix is the row-major A^T (n x m, ld)
      if (op.f64) {
        double* a = c->arena.alloc<double>((size_t)m * n);
        transpose_rect<double>((const double*)Am->val, n, m, Am->ld, a, n, s);
        op.val = a;
      } else {
        float* a = c->arena.alloc<float>((size_t)m * n);
        transpose_rect<float>((const float*)Am->val, n, m, Am->ld, a, n, s);
        op.val = a;
      }
      op.ld = n;
    }
    const size_t vs = op.f64 ? 8 : 4;
    if (op.csr) {
      op.row_ptr = Am->row_ptr;
      op.col_idx = Am->col_idx;
      {
        int* bad = c->arena.alloc<int>(1);
        const int code = check_csr(Am->row_ptr, Am->col_idx, m, n, Am->nnz, bad, s);
        APL_REQUIRE(code == 0, code & 1 ? "CSR row_ptr is malformed" : "CSR col_idx out of range");
      }
      int* tp = c->arena.alloc<int>(n + 1);
      int* ti = c->arena.alloc<int>(Am->nnz);
      void* tv = c->arena.alloc<char>(vs * (size_t)Am->nnz);
      int* scratch = c->arena.alloc<int>(n);
      if (op.f64)
        launch_csr_transpose<double>(Am->row_ptr, Am->col_idx, (const double*)Am->val, m, n, Am->nnz, tp, ti,
                                     (double*)tv, scratch, s);
      else
        launch_csr_transpose<float>(Am->row_ptr, Am->col_idx, (const float*)Am->val, m, n, Am->nnz, tp, ti,
                                    (float*)tv, scratch, s);
      op.t_ptr = tp;
      op.t_idx = ti;
      op.t_val = tv;
      op.nnz = Am->nnz;
      op.stream_t = stream_t(Am->nnz);
      // sized for the smallest tile the autotuner may pick
      int* rbA = c->arena.alloc<int>(row_block_words(Am->nnz, kTileT[0]));
      int* rbT = c->arena.alloc<int>(row_block_words(Am->nnz, kTileT[0]));
      build_row_blocks(Am->row_ptr, m, Am->nnz, op.stream_t, rbA, s);
      build_row_blocks(tp, n, Am->nnz, op.stream_t, rbT, s);
      // LDS-resident A x when x fits one workgroup's LDS (FP64 vectors need n <= about 19900)
      {
        const int tl = lx_stream_t(Am->nnz);
        int* rbL = c->arena.alloc<int>(row_block_words(Am->nnz, tl));
        build_row_blocks(Am->row_ptr, m, Am->nnz, tl, rbL, s);
        op.lx_rb = rbL;
        op.lx_grid = stream_blocks(Am->nnz, tl);
      }
      // SELL-64 copy for it when padding the 64-row slices adds at most a quarter
      if (Am->nnz >= kLxMinNnz && n * 4 <= kLxMaxBytes) {
        const long long ns = (m + 63) / 64;
        int* wid = c->arena.alloc<int>(ns);
        std::vector<int> wh;
        long long padded = sell_widths(Am->row_ptr, m, wid, wh, s);
        // one width for all slices when that pads by at most 1/32: the kernel
        // then computes each slice's offset instead of loading it
        const int wmax = wh.empty() ? 0 : *std::max_element(wh.begin(), wh.end());
        const long long upad = ns * 64 * (long long)wmax;
        int uw = 0;
        if (wmax > 0 && upad <= Am->nnz + Am->nnz / 32 && upad < (1LL << 31)) {
          uw = wmax;
          std::fill(wh.begin(), wh.end(), wmax);
          padded = upad;
        }
        if (padded <= Am->nnz + Am->nnz / 4 && padded < (1LL << 31)) {
          std::vector<int> offh(ns);
          long long acc = 0;
          for (long long i = 0; i < ns; ++i) {
            offh[i] = (int)acc;
            acc += (long long)wh[i] * 64;
          }
          int* off = c->arena.alloc<int>(ns);
          APL_HIP(hipMemcpyAsync(off, offh.data(), sizeof(int) * ns, hipMemcpyHostToDevice, s));
          if (uw > 0) APL_HIP(hipMemcpyAsync(wid, wh.data(), sizeof(int) * ns, hipMemcpyHostToDevice, s));
          int* sci = c->arena.alloc<int>(std::max<long long>(1, padded));
          void* sval = c->arena.alloc<char>(vs * (size_t)std::max<long long>(1, padded));
          if (op.f64)
            sell_fill<double>(Am->row_ptr, Am->col_idx, (const double*)Am->val, m, off, wid, sci, (double*)sval, s);
          else
            sell_fill<float>(Am->row_ptr, Am->col_idx, (const float*)Am->val, m, off, wid, sci, (float*)sval, s);
          APL_HIP(hipStreamSynchronize(s));  // offh is pageable host memory
          op.sell_off = off;
          op.sell_w = wid;
          op.sell_ci = sci;
          op.sell_val = sval;
          op.sell_slices = (int)ns;
          op.sell_uw = uw;
          op.sell_padded = padded;
          sell_layout(ns, n, &op.sell_spw, &op.sell_grid);
        }
      }
      op.rb = rbA;
      op.t_rb = rbT;
      op.group = group_for((double)Am->nnz / (double)m);
      op.t_group = group_for((double)Am->nnz / (double)n);
    } else {
      op.chunks = dense_chunks(m, n);
      op.part = c->arena.alloc<double>((size_t)std::min(1024, 4 * op.chunks) * n);
    }
    if (o->precision >= 1) {
      // FP32 copy of the values (the CSR structure is shared)
      c->fp32 = true;
      c->bf16 = o->precision == 2;
      c->op32 = op;
      c->op32.f64 = 0;
      if (op.f64) {
        if (op.csr) {
          float* v32 = c->arena.alloc<float>(Am->nnz);
          float* t32 = c->arena.alloc<float>(Am->nnz);
          to_f32((const double*)op.val, 0, v32, 0, 1, Am->nnz, s);
          to_f32((const double*)op.t_val, 0, t32, 0, 1, Am->nnz, s);
          c->op32.val = v32;
          c->op32.t_val = t32;
          if (op.sell_val) {
            float* s32 = c->arena.alloc<float>(std::max<long long>(1, op.sell_padded));
            to_f32((const double*)op.sell_val, 0, s32, 0, 1, op.sell_padded, s);
            c->op32.sell_val = s32;
          }
        } else {
          float* a32 = c->arena.alloc<float>((size_t)m * n);
          to_f32((const double*)op.val, op.ld, a32, n, m, n, s);
          c->op32.val = a32;
          c->op32.ld = n;
        }
      }
      c->u_top32 = c->arena.alloc<float>(m);
      c->u_bot32 = c->arena.alloc<float>(n);
      c->v32 = c->arena.alloc<float>(n);
      c->w32 = c->arena.alloc<float>(n);
      c->y32 = c->arena.alloc<float>(n);
      c->t32 = c->arena.alloc<float>(n);
      c->g32 = c->arena.alloc<float>(std::max(m, n));
    }
    // LSQR vectors and state
    c->u_top = c->arena.alloc<double>(m);
    c->u_bot = c->arena.alloc<double>(n);
    c->v = c->arena.alloc<double>(n);
    c->w = c->arena.alloc<double>(n);
    c->y = c->arena.alloc<double>(n);
    c->t = c->arena.alloc<double>(n);
    c->g = c->arena.alloc<double>(std::max(m, n));
    {
      const long long parts = 16384 + 256 + (op.csr ? stream_blocks(Am->nnz, kTileT[0]) : 0);
      c->wk.alpha_part = c->arena.alloc<double>(parts);
      c->wk.beta_part = c->arena.alloc<double>(parts);
    }
    c->st = c->arena.alloc<GKState>(2);
    c->counter = c->arena.alloc<unsigned>(4);
    c->st_mv = c->arena.alloc<GKState>(2);
    APL_HIP(hipMemsetAsync(c->counter, 0, 4 * sizeof(unsigned), s));
    {
      SyncGuard g(g_capture_mu);
      APL_HIP(hipHostMalloc((void**)&c->st_host, 2 * sizeof(GKState), hipHostMallocDefault));
    }
    {
      GKState& h = c->st_host[0];
      std::memset(&h, 0, sizeof(h));
      h.alpha = h.beta = h.pnorm = 1.0;
      h.nu = INFINITY;
      c->st_host[1] = h;
      APL_HIP(hipMemcpyAsync(c->st_mv, c->st_host, 2 * sizeof(GKState), hipMemcpyHostToDevice, s));
      APL_HIP(hipStreamSynchronize(s));
    }
    if (o->tune) tune_tiles(*c, s);
    if (o->precond) {
      // sketch dimensions (Alg. 3: s = ceil(1.1 b), xi' = min(xi, s), xi = 8 by default)
      int s_rows = (int)std::ceil(1.1 * o->block - 1e-12);
      s_rows = (int)std::max<long long>(1, std::min<long long>(s_rows, m));
      c->s = s_rows;
      c->xi = std::min(o->xi > 0 ? o->xi : 8, s_rows);
      c->r = o->r_probes;
      long long Lmax = std::min<long long>(std::min(m, n), 4096);
      if (o->max_rank > 0) Lmax = std::min<long long>(std::min(m, n), o->max_rank);
      c->L = (int)Lmax;
      const int jw2 = 2 * jacobi_block_width();
      c->Lpad = ((c->L + jw2 - 1) / jw2) * jw2;
      c->bmax = std::min(o->block, c->s);
      const int L = c->L, Lp = c->Lpad, b = c->bmax, S = c->s, r = c->r;
      c->S_rows = c->arena.alloc<uint16_t>((size_t)m * c->xi);
      c->S_neg = c->arena.alloc<uint8_t>(m);
      c->Y = c->arena.alloc<double>((size_t)S * n);
      c->E = c->arena.alloc<double>((size_t)S * n);
      c->W = c->arena.alloc<double>((size_t)n * r);
      c->EW = c->arena.alloc<double>((size_t)S * r);
      c->rho_dev = c->arena.alloc<double>(4);
      launch_gen_probes(o->seed, n, r, c->W, s);
      if (o->sketch >= 1) {
        // Gaussian S (s x m, column-major) in transient memory, Y = S A
        const size_t sm = (size_t)S * m;
        bool owned = false;
        char* tb = (char*)c->arena.transient(sizeof(double) * sm, owned);
        double* Sg = (double*)tb;
        launch_gen_gauss_sketch(o->seed, S, m, Sg, s);
        if (op.csr) {
          if (op.f64)
            launch_sketch_gauss_csr<double>(op.t_ptr, op.t_idx, (const double*)op.t_val, n, S, Sg, c->Y, s);
          else
            launch_sketch_gauss_csr<float>(op.t_ptr, op.t_idx, (const float*)op.t_val, n, S, Sg, c->Y, s);
        } else if (op.f64) {
          // Y^T (n x s, column-major) = A_cm (n x m) S^T: A row-major is column-major n x m with ld
          gemm(*c, Op::N, Op::T, n, S, m, 1.0, (const double*)op.val, op.ld, Sg, S, 0.0, c->Y, n);
        } else {
          // FP32 A: the product with FP32 (sketch 1) or BF16 (sketch 2) inputs on
          // MFMA, chunk sums accumulated in FP64
          sketch_gemm_f32((const float*)op.val, m, n, op.ld, Sg, S, c->Y, o->sketch == 2, s);
        }
        APL_HIP(hipStreamSynchronize(s));
        if (owned) {
          SyncGuard g(g_capture_mu);
          APL_HIP(hipFree(tb));
        }
      } else if (op.csr) {
        launch_gen_sketch(o->seed, S, m, c->xi, c->S_rows, c->S_neg, s);
        if (op.f64)
          launch_sketch_csr<double>(op.t_ptr, op.t_idx, (const double*)op.t_val, n, S, c->xi, c->S_rows,
                                    c->S_neg, c->Y, s);
        else
          launch_sketch_csr<float>(op.t_ptr, op.t_idx, (const float*)op.t_val, n, S, c->xi, c->S_rows,
                                   c->S_neg, c->Y, s);
      } else {
        launch_gen_sketch(o->seed, S, m, c->xi, c->S_rows, c->S_neg, s);
        bool owned = false;
        void* part = c->arena.transient(sketch_dense_scratch(m, S, c->xi), owned);
        if (op.f64)
          launch_sketch_dense<double>((const double*)op.val, m, n, op.ld, S, c->xi, c->S_rows, c->S_neg, c->Y,
                                      part, s);
        else
          launch_sketch_dense<float>((const float*)op.val, m, n, op.ld, S, c->xi, c->S_rows, c->S_neg, c->Y,
                                     part, s);
        APL_HIP(hipStreamSynchronize(s));
        if (owned) {
          SyncGuard g(g_capture_mu);
          APL_HIP(hipFree(part));
        }
      }
      // CUR / preconditioner storage (sized by the rank cap L)
      c->I_dev = c->arena.alloc<int>(L);
      c->J_dev = c->arena.alloc<int>(L);
      c->Ip = c->arena.alloc<int>(b);
      c->Jp = c->arena.alloc<int>(S);
      c->C = c->arena.alloc<double>((size_t)m * L);
      c->Rt = c->arena.alloc<double>((size_t)n * L);
      c->U = c->arena.alloc<double>((size_t)L * L);
      c->Q = c->arena.alloc<double>((size_t)n * L);
      c->TR = c->arena.alloc<double>((size_t)L * L);
      c->TC = c->arena.alloc<double>((size_t)L * L);
      c->Ecol = c->arena.alloc<double>((size_t)m * b);
      c->RJ = c->arena.alloc<double>((size_t)S * L);
      c->F = c->arena.alloc<double>((size_t)L * S);
      c->Gm = c->arena.alloc<double>((size_t)b * L);
      c->H = c->arena.alloc<double>((size_t)b * L);
      c->B21 = c->arena.alloc<double>((size_t)b * L);
      c->Sb = c->arena.alloc<double>((size_t)b * b);
      c->Sinv = c->arena.alloc<double>((size_t)b * b);
      c->lu_piv = c->arena.alloc<int>(b);
      c->small = c->arena.alloc<double>((size_t)4 * b * b);
      // Y(:, J) and Z = Y(:, J) U with an even leading dimension, so that
      // the GEMMs read them with 16-byte loads
      c->YJ = c->arena.alloc<double>((size_t)(S + (S & 1)) * L);
      c->Z = c->arena.alloc<double>((size_t)(S + (S & 1)) * L);
      c->P2 = c->arena.alloc<double>((size_t)L * b);
      c->status_dev = c->arena.alloc<int>(4);
      c->Mx = c->arena.alloc<double>((size_t)L * Lp);
      c->Vm = c->arena.alloc<double>((size_t)Lp * Lp);
      c->sigma = c->arena.alloc<double>(Lp);
      c->Kc = c->arena.alloc<double>((size_t)L * L);
      c->Kr = c->arena.alloc<double>((size_t)L * L);
      c->d = c->arena.alloc<double>(L);
      c->pinfo = c->arena.alloc<double>(4);
      if (c->o.precond != 2) c->jac_part = c->arena.alloc<double>((size_t)jacobi_work_words(Lp));
      c->pa_c = c->arena.alloc<double>(L);
      c->prec.c = c->pa_c;
      c->prec.d = c->d;
      if (op.csr && c->o.precond != 2) {
        // implicit P-apply: R = A(I,:) and its transpose, capacity nnz(A)
        c->prec.implicit = 1;
        c->rr_ptr = c->arena.alloc<int>(L + 1);
        c->rr_idx = c->arena.alloc<int>(Am->nnz);
        c->rr_val = c->arena.alloc<double>(Am->nnz);
        c->rt_ptr = c->arena.alloc<int>(n + 1);
        c->rt_idx = c->arena.alloc<int>(Am->nnz);
        c->rt_val = c->arena.alloc<double>(Am->nnz);
        c->rscratch = c->arena.alloc<int>(std::max<long long>(n, L));
        c->pc1 = c->arena.alloc<double>(L);
        c->pc2 = c->arena.alloc<double>(L);
        c->M2 = c->arena.alloc<double>((size_t)L * L);
        c->prec.I = c->I_dev;
        c->prec.Kt = c->Kc;
        c->prec.Kr = c->Kr;
        c->prec.rt_ptr = c->rt_ptr;
        c->prec.rt_idx = c->rt_idx;
        c->prec.rt_val = c->rt_val;
        c->prec.c1 = c->pc1;
        c->prec.c2 = c->pc2;
      } else {
        // explicit P-apply through V (n x l): always for a dense A, and for the
        // SVD-free form, whose non-normal middle factor would amplify the
        // rounding of I - Q_R Q_R^T formed through Q_R = R^T T_R^{-1}
        c->prec.implicit = 0;
        c->Vhat = c->arena.alloc<double>((size_t)L * n);
        const int pchunks = (int)std::max<long long>(1, std::min<long long>(256, n / 64));
        c->pa_part = c->arena.alloc<double>((size_t)pchunks * L);
        c->prec.chunks = pchunks;
        c->prec.part = c->pa_part;
        c->prec.V = c->Vhat;
        if (c->o.precond == 2) {
          c->M2 = c->arena.alloc<double>((size_t)L * L);
          c->M2t = c->arena.alloc<double>((size_t)L * L);
          c->pc2 = c->arena.alloc<double>(L);
          c->prec.c2 = c->pc2;
        }
      }
      long long lrows = std::max(m, n);
      c->fw.lupp_rows = (int)lrows;
      c->fw.pos = c->arena.alloc<int>(2 * lrows);
      c->fw.row_at = c->arena.alloc<int>(2 * lrows);
      c->fw.pv = c->arena.alloc<double>(2048);
      c->fw.pp = c->arena.alloc<int>(2048);
      c->fw.pi = c->arena.alloc<int>(2048);
      c->fw.lupp_state = c->arena.alloc<int>(4);
      c->fw.lupp_g = c->arena.alloc<double>((size_t)kLuppNB * (std::max(c->s, b) + 8));
      c->fw.counter = c->counter + 1;
      fill(c->TR, (long long)L * L, 0.0, s);
      fill(c->TC, (long long)L * L, 0.0, s);
      fill(c->U, (long long)L * L, 0.0, s);
    }
    APL_HIP(hipStreamSynchronize(s));
    c->t_sketch = ms_since(t0);
    return c;
  } catch (...) {
    delete c;
    throw;
  }
}

// ------------------------------------------------------------------ LU pivots (Alg. 7)
// First k partial-pivoting pivots of X (r x cols, column-major, ld), panel by
// panel: within a panel of kLuppNB pivots the steps eliminate only the panel's
// columns; the trailing columns are then updated at once (U12 = L11^{-1} A12 on
// the panel's pivot rows, X(:, trail) -= X(:, panel) U12), which is the same
// elimination in another summation order.  Pivot rows are never read again, so
// the update runs over all rows.
static void lupp_blocked(Ctx& c, double* X, int r, int cols, long long ld, int k, int* piv, hipStream_t s) {
  lupp_begin(X, r, k, c.fw, s);
  for (int q0 = 0; q0 < k; q0 += kLuppNB) {
    const int qe = std::min(q0 + kLuppNB, k);
    for (int q = q0; q < qe; ++q) lupp_step(X, r, cols, qe, ld, q, k, piv, c.fw, s);
    if (qe >= k || qe >= cols) break;
    const int nb = qe - q0, w = cols - q0;
    double* G = c.fw.lupp_g;
    lupp_gather(X, r, ld, piv, q0, nb, w, G, s);
    trsm(c, Side::Left, Uplo::Lower, Op::N, Diag::Unit, nb, cols - qe, 1.0, G, nb, G + (size_t)nb * nb, nb);
    gemm(c, Op::N, Op::N, r, cols - qe, nb, -1.0, X + (long long)q0 * ld, ld,
         G + (size_t)nb * nb, nb, 1.0, X + (long long)qe * ld, ld);
    lupp_cand(X, r, ld, qe, c.fw, s);
  }
}

// ------------------------------------------------------------------ small dense factorisations
// Upper Cholesky G = U^T U of the k x k SPD matrix G (column-major, ld) in
// place, the strict lower triangle cleared; status_dev[0] != 0 on failure.
// Blocked: diagonal blocks in LDS (one workgroup), TRSM and SYRK for the rest.
static void chol_upper(Ctx& c, double* G, long long ld, int k, hipStream_t s) {
  APL_HIP(hipMemsetAsync(c.status_dev, 0, sizeof(int), s));
  for (int j0 = 0; j0 < k; j0 += kFNB) {
    const int nb = std::min(kFNB, k - j0), r = k - j0 - nb;
    double* D = G + j0 + (long long)j0 * ld;
    potrf_diag(D, ld, nb, j0, c.status_dev, s);
    if (r > 0) {
      double* G12 = G + j0 + (long long)(j0 + nb) * ld;
      trsm(c, Side::Left, Uplo::Upper, Op::T, Diag::NonUnit, nb, r, 1.0, D, ld, G12, ld);
      // trailing update G22 -= G12^T G12 (both triangles; the lower one is cleared at the end)
      gemm(c, Op::T, Op::N, r, r, nb, -1.0, G12, ld, G12, ld, 1.0, G + (j0 + nb) + (long long)(j0 + nb) * ld, ld);
    }
  }
  zero_lower(G, ld, k, s);
}

// Sinv = S^{-1} for the k x k matrix S (column-major, ld; overwritten by its
// LU factors): blocked LU with partial pivoting (panels in LDS, TRSM and GEMM
// for the trailing matrix), then Sinv = U^{-1} L^{-1} P.  status_dev[0] = 1 if
// S is singular.
static void lu_inverse(Ctx& c, double* S, long long ld, int k, double* Sinv, long long ldi, hipStream_t s) {
  APL_HIP(hipMemsetAsync(c.status_dev, 0, sizeof(int), s));
  for (int j0 = 0; j0 < k; j0 += kFNB) {
    const int w = std::min(kFNB, k - j0), r = k - j0 - w;
    lu_panel(S, ld, k, j0, w, c.lu_piv, c.status_dev, s);
    laswp(S, ld, k, j0, j0 + w, c.lu_piv, j0, w, s);
    if (r > 0) {
      double* A12 = S + j0 + (long long)(j0 + w) * ld;
      trsm(c, Side::Left, Uplo::Lower, Op::N, Diag::Unit, w, r, 1.0, S + j0 + (long long)j0 * ld, ld, A12, ld);
      gemm(c, Op::N, Op::N, r, r, w, -1.0, S + (j0 + w) + (long long)j0 * ld, ld,
           A12, ld, 1.0, S + (j0 + w) + (long long)(j0 + w) * ld, ld);
    }
  }
  set_identity(Sinv, ldi, k, s);
  laswp(Sinv, ldi, k, 0, 0, c.lu_piv, 0, k, s);
  trsm(c, Side::Left, Uplo::Lower, Op::N, Diag::Unit, k, k, 1.0, S, ld, Sinv, ldi);
  trsm(c, Side::Left, Uplo::Upper, Op::N, Diag::NonUnit, k, k, 1.0, S, ld, Sinv, ldi);
}

// ------------------------------------------------------------------ Cholesky QR
// X (n x k, column-major ld) <- Q, R (k x k upper, ldr) with X_in = Q R, by
// Cholesky QR applied twice (a shift is added to the first Gram matrix if
// its Cholesky factorisation fails: shifted CholeskyQR, Fukaya et al.).
static void chol_qr2(Ctx& c, double* X, long long n, int k, long long ldx, double* R, long long ldr, hipStream_t s) {
  double* G = c.small;                             // k x k
  double* R1 = c.small + (size_t)c.bmax * c.bmax;  // k x k
  double* Racc = c.small + 2 * (size_t)c.bmax * c.bmax;
  int passes = 2;
  for (int pass = 0; pass < passes; ++pass) {
    gemm(c, Op::T, Op::N, k, k, n, 1.0, X, ldx, X, ldx, 0.0, G, k);
    chol_upper(c, G, k, k, s);
    if (read_int(c.status_dev, s) != 0) {
      APL_REQUIRE(pass == 0, "Cholesky QR failed (block numerically rank deficient)");
      // shifted Cholesky QR: G + shift I, then one extra unshifted pass
      gemm(c, Op::T, Op::N, k, k, n, 1.0, X, ldx, X, ldx, 0.0, G, k);
      std::vector<double> hg((size_t)k * k);
      APL_HIP(hipMemcpyAsync(hg.data(), G, sizeof(double) * k * k, hipMemcpyDeviceToHost, s));
      APL_HIP(hipStreamSynchronize(s));
      double dmax = 0.0;
      for (int i = 0; i < k; ++i) dmax = std::max(dmax, hg[(size_t)i * k + i]);
      const double shift = 11.0 * 2.2e-16 * (double)(n * k + (long long)k * (k + 1)) * std::max(dmax, 1e-300);
      for (int i = 0; i < k; ++i) hg[(size_t)i * k + i] += shift;
      APL_HIP(hipMemcpyAsync(G, hg.data(), sizeof(double) * k * k, hipMemcpyHostToDevice, s));
      chol_upper(c, G, k, k, s);
      APL_REQUIRE(read_int(c.status_dev, s) == 0, "shifted Cholesky QR failed");
      passes = 3;
    }
    trsm(c, Side::Right, Uplo::Upper, Op::N, Diag::NonUnit, n, k, 1.0, G, k, X, ldx);
    if (pass == 0) {
      copy_block(G, k, Racc, k, k, k, 1.0, s);
    } else {
      gemm(c, Op::N, Op::N, k, k, k, 1.0, G, k, Racc, k, 0.0, R1, k);
      copy_block(R1, k, Racc, k, k, k, 1.0, s);
    }
  }
  copy_block(Racc, k, R, ldr, k, k, 1.0, s);
}

// ------------------------------------------------------------------ one outer step
// ------------------------------------------------------------------ T_C by sketched Cholesky QR
// Stream offset of the embedding Theta below: the Gaussian embedding of seed
// + kTcSeedOffset (stream 3), never the Gaussian sketch of A.
constexpr uint64_t kTcSeedOffset = 7919;

// T_C(0:ln, 0:ln) by sketched Cholesky QR of C(:, 0:ln), the stable choice
// Alg. 2 and Alg. 3 Part 3 name for T_C, used when chol(C^T C) breaks down:
// Theta (k x m Gaussian, k = min(m, 2 ln)), X = Theta C; two shifted passes
// R_i = chol(X^T X + s I), s = 11 (k ln + ln (ln + 1)) u ||X||_F^2, and two
// plain passes R_i = chol(X^T X), each followed by X <- X R_i^{-1}; R = R_4 R_3
// R_2 R_1; Q = C R^{-1}; T_C = chol(Q^T Q) R.  Returns false (T_C untouched)
// when a Cholesky breaks down or the transient memory is not available.
static bool tc_sketched(Ctx& c, int ln, hipStream_t s) {
  const long long m = c.m;
  const int k = (int)std::min<long long>(m, 2LL * ln);
  const size_t nTh = (size_t)k * m, nX = (size_t)k * ln, nQ = (size_t)m * ln, nR = (size_t)ln * ln;
  const size_t parts[6] = {nTh, nX, nQ, nR, nR, nR};
  size_t bytes = 0;
  for (size_t p : parts) bytes += Arena::aligned(sizeof(double) * p);
  bool owned = false;
  char* tb = nullptr;
  try {
    tb = (char*)c.arena.transient(bytes, owned);
  } catch (const Error&) {
    return false;
  }
  double* ptr[6];
  {
    char* q = tb;
    for (int i = 0; i < 6; ++i) {
      ptr[i] = (double*)q;
      q += Arena::aligned(sizeof(double) * parts[i]);
    }
  }
  double *Th = ptr[0], *X = ptr[1], *Q = ptr[2], *G = ptr[3], *R = ptr[4], *Rt = ptr[5];
  bool ok = true;
  launch_gen_gauss_sketch(c.o.seed + kTcSeedOffset, k, m, Th, s);
  gemm(c, Op::N, Op::N, k, ln, m, 1.0, Th, k, c.C, m, 0.0, X, k);
  set_identity(R, ln, ln, s);
  for (int pass = 0; pass < 4 && ok; ++pass) {
    gemm(c, Op::T, Op::N, ln, ln, k, 1.0, X, k, X, k, 0.0, G, ln);
    if (pass < 2) {
      const double nf = dnrm2((long long)k * ln, X, c.nrm_tmp, s);
      add_diag(G, ln, ln, 11.0 * ((double)k * ln + (double)ln * (ln + 1)) * 0x1p-53 * nf * nf, s);
    }
    chol_upper(c, G, ln, ln, s);
    if (read_int(c.status_dev, s) != 0) {
      ok = false;
      break;
    }
    trsm(c, Side::Right, Uplo::Upper, Op::N, Diag::NonUnit, k, ln, 1.0, G, ln, X, k);
    gemm(c, Op::N, Op::N, ln, ln, ln, 1.0, G, ln, R, ln, 0.0, Rt, ln);
    std::swap(R, Rt);
  }
  if (ok) {
    copy_block(c.C, m, Q, m, (int)m, ln, 1.0, s);
    trsm(c, Side::Right, Uplo::Upper, Op::N, Diag::NonUnit, m, ln, 1.0, R, ln, Q, m);
    gemm(c, Op::T, Op::N, ln, ln, m, 1.0, Q, m, Q, m, 0.0, G, ln);
    chol_upper(c, G, ln, ln, s);
    if (read_int(c.status_dev, s) != 0) ok = false;
  }
  if (ok) {
    gemm(c, Op::N, Op::N, ln, ln, ln, 1.0, G, ln, R, ln, 0.0, Rt, ln);
    zero_lower(Rt, ln, ln, s);
    copy_block(Rt, ln, c.TC, c.L, ln, ln, 1.0, s);
  }
  APL_HIP(hipStreamSynchronize(s));
  if (owned) {
    SyncGuard g(g_capture_mu);
    APL_HIP(hipFree(tb));
  }
  return ok;
}

struct StepResult {
  double rho;
  bool exhausted;
  int added;
};

static StepResult outer_step(Ctx& c, hipStream_t s) {
  const long long m = c.m, n = c.n;
  const int S = c.s, L = c.L, l = c.rank;
  StepResult res{0.0, false, 0};
  int beff = std::min<long long>(std::min<long long>(c.bmax, n - l), std::min<long long>(m - l, L - l));
  if (beff <= 0) {
    res.exhausted = true;
    res.rho = c.rho_hist.empty() ? 0.0 : c.rho_hist.back();
    return res;
  }
  // (i)-(ii) column pivots from the sketched residual (E_row^T = E as n x s column-major)
  if (l > 0) zero_rows(c.E, n, c.J_dev, l, S, s);
  lupp_blocked(c, c.E, (int)n, S, n, beff, c.Jp, s);
  const int k1 = lupp_read_keff(c.fw, s);
  if (k1 == 0) {
    res.exhausted = true;
    res.rho = c.rho_hist.empty() ? 0.0 : c.rho_hist.back();
    return res;
  }
  // (iii) new columns of C and the column residual E_col = A(:,J+) - C U R(:,J+)
  double* Cn = c.C + (size_t)l * m;
  gather_cols(c.op, c.Jp, k1, Cn, m, s);
  copy_block(Cn, m, c.Ecol, m, (int)m, k1, 1.0, s);
  if (l > 0) {
    gather_sub_rows(c.Rt, n, c.Jp, k1, l, c.RJ, k1, s);  // RJ = R(:,J+)^T, k1 x l
    gemm(c, Op::N, Op::T, l, k1, l, 1.0, c.U, L, c.RJ, k1, 0.0, c.F, L);
    gemm(c, Op::N, Op::N, m, k1, l, -1.0, c.C, m, c.F, L, 1.0, c.Ecol, m);
    zero_rows(c.Ecol, m, c.I_dev, l, k1, s);
  }
  // (iv) row pivots of E_col
  lupp_blocked(c, c.Ecol, (int)m, k1, m, k1, c.Ip, s);
  const int k2 = lupp_read_keff(c.fw, s);
  if (k2 < beff) res.exhausted = true;
  if (k2 == 0) {
    res.rho = c.rho_hist.empty() ? 0.0 : c.rho_hist.back();
    return res;
  }
  std::vector<int> hJ(k2), hI(k2);
  APL_HIP(hipMemcpyAsync(hJ.data(), c.Jp, sizeof(int) * k2, hipMemcpyDeviceToHost, s));
  APL_HIP(hipMemcpyAsync(hI.data(), c.Ip, sizeof(int) * k2, hipMemcpyDeviceToHost, s));
  APL_HIP(hipMemcpyAsync(c.J_dev + l, c.Jp, sizeof(int) * k2, hipMemcpyDeviceToDevice, s));
  APL_HIP(hipMemcpyAsync(c.I_dev + l, c.Ip, sizeof(int) * k2, hipMemcpyDeviceToDevice, s));
  APL_HIP(hipStreamSynchronize(s));
  c.J.insert(c.J.end(), hJ.begin(), hJ.end());
  c.I.insert(c.I.end(), hI.begin(), hI.end());
  // new rows of R (as columns of Rt)
  double* Rn = c.Rt + (size_t)l * n;
  gather_rows(c.op, c.Ip, k2, Rn, n, s);
  // (v) U = A(I,J)^{-1} by the block-inverse update; Schur complement
  //     S = A(I+,J+) - A(I+,J) U A(I,J+)
  gather_sub_rows(Cn, m, c.Ip, k2, k2, c.Sb, k2, s);  // A(I+, J+)
  if (l > 0) {
    gather_sub_rows(c.C, m, c.Ip, k2, l, c.B21, k2, s);  // A(I+, J_old), k2 x l
    gemm(c, Op::N, Op::N, k2, l, l, 1.0, c.B21, k2, c.U, L, 0.0, c.Gm, k2);
    // S -= G B12, B12 = RJ(0:k2, :)^T
    gemm(c, Op::N, Op::T, k2, k2, l, -1.0, c.Gm, k2, c.RJ, k1, 1.0, c.Sb, k2);
  }
  lu_inverse(c, c.Sb, k2, k2, c.Sinv, k2, s);
  if (read_int(c.status_dev, s) != 0) throw Error(APLICUR_E_BREAKDOWN, "singular CUR core block");
  if (l == 0) {
    copy_block(c.Sinv, k2, c.U, L, k2, k2, 1.0, s);
  } else {
    gemm(c, Op::N, Op::N, k2, l, k2, 1.0, c.Sinv, k2, c.Gm, k2, 0.0, c.H, k2);
    gemm(c, Op::N, Op::N, l, l, k2, 1.0, c.F, L, c.H, k2, 1.0, c.U, L);
    gemm(c, Op::N, Op::N, l, k2, k2, -1.0, c.F, L, c.Sinv, k2, 0.0,
         c.U + (size_t)l * L, L);
    copy_block(c.H, k2, c.U + l, L, k2, l, -1.0, s);
    copy_block(c.Sinv, k2, c.U + l + (size_t)l * L, L, k2, k2, 1.0, s);
  }
  const int ln = l + k2;
  // (vi) E_row = Y - (Y(:,J) U) R   (E as n x s column-major = E_row^T)
  const int Sp = S + (S & 1);  // leading dimension of YJ and Z
  gather_y_cols(c.Y, n, S, c.J_dev, ln, c.YJ, Sp, s);
  gemm(c, Op::N, Op::N, S, ln, ln, 1.0, c.YJ, Sp, c.U, L, 0.0, c.Z, Sp);
  APL_HIP(hipMemcpyAsync(c.E, c.Y, sizeof(double) * (size_t)S * n, hipMemcpyDeviceToDevice, s));
  gemm(c, Op::N, Op::T, n, S, ln, -1.0, c.Rt, n, c.Z, Sp, 1.0, c.E, n);
  // (vii) rho = 10 sqrt(2/pi) max_i ||E_row w_i||
  gemm(c, Op::T, Op::N, S, c.r, n, 1.0, c.E, n, c.W, n, 0.0, c.EW, S);
  rho_from_ew(c.EW, S, c.r, c.rho_dev, s);
  // (viii) augmentQR (Alg. 9) with the new columns A(I+,:)^T
  double* Qn = c.Q + (size_t)l * n;
  copy_block(Rn, n, Qn, n, (int)n, k2, 1.0, s);
  if (l > 0) {
    double* P1 = c.TR + (size_t)l * L;  // T_R(0:l, l:ln)
    gemm(c, Op::T, Op::N, l, k2, n, 1.0, c.Q, n, Rn, n, 0.0, P1, L);
    gemm(c, Op::N, Op::N, n, k2, l, -1.0, c.Q, n, P1, L, 1.0, Qn, n);
    gemm(c, Op::T, Op::N, l, k2, n, 1.0, c.Q, n, Qn, n, 0.0, c.P2, l);
    gemm(c, Op::N, Op::N, n, k2, l, -1.0, c.Q, n, c.P2, l, 1.0, Qn, n);
    // P1 += P2
    add_block(c.P2, l, P1, L, l, k2, s);
  }
  chol_qr2(c, Qn, n, k2, n, c.TR + l + (size_t)l * L, L, s);
  // (ix) T_C = chol(C^T C), extended: T12 = T_C^{-T} C_old^T C_new, T22 = chol(C_new^T C_new - T12^T T12);
  //      when that Cholesky breaks down, the whole T_C by sketched Cholesky QR (option tc_sketched)
  {
    double* T12 = c.TC + (size_t)l * L;
    double* T22 = c.TC + l + (size_t)l * L;
    if (l > 0) {
      gemm(c, Op::T, Op::N, l, k2, m, 1.0, c.C, m, Cn, m, 0.0, T12, L);
      trsm(c, Side::Left, Uplo::Upper, Op::T, Diag::NonUnit, l, k2, 1.0, c.TC, L, T12, L);
    }
    double* G22 = c.small;
    gemm(c, Op::T, Op::N, k2, k2, m, 1.0, Cn, m, Cn, m, 0.0, G22, k2);
    if (l > 0)
      gemm(c, Op::T, Op::N, k2, k2, l, -1.0, T12, L, T12, L, 1.0, G22, k2);
    chol_upper(c, G22, k2, k2, s);
    if (read_int(c.status_dev, s) == 0) {
      copy_block(G22, k2, T22, L, k2, k2, 1.0, s);
    } else if (!(c.o.tc_sketched && tc_sketched(c, ln, s))) {
      // C^T C is not positive definite in floating point (the new columns
      // are nearly dependent on C), and sketched Cholesky QR is off or
      // breaks down too.  Undo the step (U11 back to its old value; the new
      // slots of I, J, C, R, Q_R, T_R lie beyond the rank and are ignored)
      // and end the rank growth.
      if (l == 0) throw Error(APLICUR_E_BREAKDOWN, "the first CUR columns are dependent (T_C)");
      gemm(c, Op::N, Op::N, l, l, k2, -1.0, c.F, L, c.H, k2, 1.0, c.U, L);
      c.J.resize(l);
      c.I.resize(l);
      APL_HIP(hipStreamSynchronize(s));
      res.exhausted = true;
      res.added = 0;
      res.rho = c.rho_hist.empty() ? 0.0 : c.rho_hist.back();
      return res;
    }
  }
  double rho = 0.0;
  APL_HIP(hipGetLastError());
  APL_HIP(hipMemcpyAsync(&rho, c.rho_dev, sizeof(double), hipMemcpyDeviceToHost, s));
  APL_HIP(hipStreamSynchronize(s));
  c.rank = ln;
  res.rho = rho;
  res.added = k2;
  return res;
}

// ------------------------------------------------------------------ preconditioner (Alg. 2 Part 2)
// The one-sided Jacobi SVD of the core M stops when the off-diagonal of the
// Gram matrix of the damped core [M; delta I] (entries scaled to unit
// diagonal) has Frobenius norm at most jacobi_tol (option; kJacobiTol by default).  With V the accumulated
// rotations (orthogonal to rounding) and Lambda_i^2 = ||M v_i||^2 + delta^2,
// the core part of the preconditioned Gram, diag(sigma_hat / Lambda) V^T (M^T
// M + delta^2 I) V diag(sigma_hat / Lambda), is sigma_hat^2 (I + E) with that
// off-diagonal E, so its singular values lie within sqrt(1 +- jacobi_tol) of
// the exact-SVD value sigma_hat.  A block pair whose scaled entries are all
// at most skip = jacobi_tol / (4 l) (and at most kJacobiSkip) is not rotated:
// such entries still count in the stopping test, and all l^2 of them
// together are at most jacobi_tol / 4 in Frobenius norm, so skipping them
// cannot keep the sweeps from reaching the test.
constexpr double kJacobiSkip = 1e-6;
// Largest diagonal ratio of T_R for which the one-product form M2 is used.
constexpr double kM2MaxDiagRatio = 1e3;

// CSR of R = A(I,:) and of R^T (the implicit P-apply reads R^T rows).
static void build_r_csr(Ctx& c, hipStream_t s) {
  const int l = c.rank;
  long long nnzR;
  if (c.op.f64)
    nnzR = launch_gather_csr_rows<double>(c.op.row_ptr, c.op.col_idx, (const double*)c.op.val, c.I_dev, l, c.rr_ptr,
                                          c.rr_idx, c.rr_val, c.op.nnz, c.rscratch, s);
  else
    nnzR = launch_gather_csr_rows<float>(c.op.row_ptr, c.op.col_idx, (const float*)c.op.val, c.I_dev, l, c.rr_ptr,
                                         c.rr_idx, c.rr_val, c.op.nnz, c.rscratch, s);
  launch_csr_transpose<double>(c.rr_ptr, c.rr_idx, c.rr_val, l, c.n, nnzR, c.rt_ptr, c.rt_idx, c.rt_val, c.rscratch,
                               s);
}

// SVD-free preconditioner (Alg. 8, the SVD-free variant of Sec. 3.1; mu = 0):
//   P~^{-1} = t Q_R M^{-1} Q_R^T + (I - Q_R Q_R^T),   M^{-1} = T_R^{-T} A(I,J) T_C^{-1},
// with target level t = max(rho, eps_cur), rho of the last CUR step (a CUR
// more accurate than eps_cur, rho at rounding level at full rank, would
// flatten the captured spectrum to a level that rounding dominates).  With
// H = t M^{-1} - I the apply is z + Q_R H Q_R^T z with the orthonormal Q_R of
// augmentQR as V (dense and CSR alike); H is formed once per build by two
// triangular solves and costs one l x l product per apply.  P~ is not
// symmetric: the transpose apply uses H^T.  ||P~|| = max(1, ||M||_2 / t) is
// bounded with ||M||_F, M = T_C U T_R^T.
static void build_precond_svdfree(Ctx& c, hipStream_t s) {
  const int l = c.rank, L = c.L;
  const double rho = c.rho_hist.empty() ? 0.0 : c.rho_hist.back();
  const double target = std::max(rho, c.eps_cur);
  gemm(c, Op::N, Op::T, l, l, l, 1.0, c.U, L, c.TR, L, 0.0, c.Kr, l);
  gemm(c, Op::N, Op::N, l, l, l, 1.0, c.TC, L, c.Kr, l, 0.0, c.Kc, l);
  double mfro = 0.0;
  mfro = dnrm2((long long)l * l, c.Kc, c.nrm_tmp, s);
  // H = target T_R^{-T} W T_C^{-1} - I with W = A(I,J) = C(I,:), column-major in Mx (ld l)
  gather_sub_rows(c.C, c.m, c.I_dev, l, l, c.Mx, l, s);
  trsm(c, Side::Right, Uplo::Upper, Op::N, Diag::NonUnit, l, l, target, c.TC, L, c.Mx, l);
  trsm(c, Side::Left, Uplo::Upper, Op::T, Diag::NonUnit, l, l, 1.0, c.TR, L, c.Mx, l);
  add_diag(c.Mx, l, l, -1.0, s);
  // V = Q_R, row-major n x l
  transpose_rect<double>(c.Q, l, c.n, c.n, c.Vhat, l, s);
  c.prec.ldv = l;
  // H (column-major in Mx) row-major for the forward apply, and H^T row-major
  // (= H column-major) for the transpose apply
  transpose_square(c.Mx, l, c.M2, l, s);
  copy_block(c.Mx, l, c.M2t, l, l, l, 1.0, s);
  c.prec.M2 = c.M2;
  c.prec.M2t = c.M2t;
  APL_HIP(hipGetLastError());
  APL_HIP(hipStreamSynchronize(s));
  c.sweep_hist.push_back(0);
  c.p_sigma_host.clear();
  c.p_sigma_l = target;
  c.p_target = target;
  c.p_pnorm = std::max(1.0, mfro / target);
  c.prec.ell = l;
  c.have_prec = true;
  ++c.prec_gen;
}

static void build_precond(Ctx& c, hipStream_t s) {
  if (c.o.precond == 2) {
    build_precond_svdfree(c, s);
    return;
  }
  const int l = c.rank, L = c.L;
  const int jw2 = 2 * jacobi_block_width();
  const int lp = ((l + jw2 - 1) / jw2) * jw2;
  // M = T_C U T_R^T  (l x l) into Mx (ld L, lp columns, padding zero)
  fill(c.Mx, (long long)L * lp, 0.0, s);
  gemm(c, Op::N, Op::T, l, l, l, 1.0, c.U, L, c.TR, L, 0.0, c.Kr, l);
  gemm(c, Op::N, Op::N, l, l, l, 1.0, c.TC, L, c.Kr, l, 0.0, c.Mx, L);
  // Warm start: the Jacobi iteration accepts any orthogonal starting basis V0
  // (it computes M V0 times rotations).  The previous build's right singular
  // vectors V_old (rank l_old) are coordinates in the leading l_old columns of
  // Q_R, which augmentQR keeps, and the dominant directions of the grown CUR
  // stay close to them; V0 = blkdiag(V_old, I) starts the sweeps nearly
  // converged in those directions.  X0 = M V0 replaces the first l_old columns.
  const int lo = (c.vm_rank > 0 && c.vm_rank < l) ? c.vm_rank : 0;
  if (lo > 0) {
    copy_block(c.Vm, c.vm_ld, c.Kc, lo, lo, lo, 1.0, s);  // V_old (lo x lo, ld lo)
    set_identity(c.Vm, lp, lp, s);
    copy_block(c.Kc, lo, c.Vm, lp, lo, lo, 1.0, s);
    gemm(c, Op::N, Op::N, l, lo, lo, 1.0, c.Mx, L, c.Kc, lo, 0.0, c.Kr, l);  // M(:, 0:lo) V_old
    copy_block(c.Kr, l, c.Mx, L, l, lo, 1.0, s);
  } else {
    set_identity(c.Vm, lp, lp, s);
  }
  c.sweep_hist.push_back(
      jacobi_svd(c.Mx, L, l, lp, c.Vm, lp, c.sigma, c.jac_part, c.delta * c.delta, c.jacobi_tol,
                 std::min(kJacobiSkip, c.jacobi_tol / (4.0 * l)), 40, s));
  c.vm_rank = l;
  c.vm_ld = lp;
  precond_scalars(c.sigma, l, c.delta, c.d, c.pinfo, s);
  if (c.prec.implicit) {
    // K = T_R^{-1} V_M (column-major, ld l: the row-major K^T) and K row-major
    copy_block(c.Vm, lp, c.Kc, l, l, l, 1.0, s);
    trsm(c, Side::Left, Uplo::Upper, Op::N, Diag::NonUnit, l, l, 1.0, c.TR, L, c.Kc, l);
    // M2 = K diag(d) K^T replaces the two K products when T_R is well
    // conditioned (its rounding error grows with cond(T_R)^2, the two-product
    // form's with cond(T_R)); the diagonal ratio of T_R is the indicator.
    std::vector<double> diag(l);
    APL_HIP(hipMemcpy2DAsync(diag.data(), sizeof(double), c.TR, (size_t)(L + 1) * sizeof(double), sizeof(double), l,
                             hipMemcpyDeviceToHost, s));
    APL_HIP(hipStreamSynchronize(s));
    double dmin = INFINITY, dmax = 0.0;
    for (double v : diag) {
      dmin = std::min(dmin, std::fabs(v));
      dmax = std::max(dmax, std::fabs(v));
    }
    if (dmin > 0.0 && dmax / dmin <= kM2MaxDiagRatio) {
      scale_cols(c.Kc, l, l, l, c.d, c.Kr, s);
      gemm(c, Op::N, Op::T, l, l, l, 1.0, c.Kr, l, c.Kc, l, 0.0, c.M2, l);
      c.prec.M2 = c.M2;
    } else {
      transpose_square(c.Kc, l, c.Kr, l, s);
      c.prec.M2 = nullptr;
    }
    build_r_csr(c, s);
  } else {
    // V = Q_R V_M (n x l row-major in Vhat) is formed by ensure_vhat for the
    // one-column paths when they first apply this P; the blocked path applies
    // Q_R and V_M diag(d) V_M^T as factors (blk_prec)
    c.vhat_kind = 0;
    c.prec.ldv = l;
  }
  double info[4];
  APL_HIP(hipMemcpyAsync(info, c.pinfo, sizeof(info), hipMemcpyDeviceToHost, s));
  c.p_sigma_host.resize(l);
  APL_HIP(hipMemcpyAsync(c.p_sigma_host.data(), c.sigma, sizeof(double) * l, hipMemcpyDeviceToHost, s));
  APL_HIP(hipStreamSynchronize(s));
  c.p_sigma_l = info[0];
  c.p_target = info[2];
  c.p_pnorm = info[3];
  c.prec.ell = l;
  c.have_prec = true;
  ++c.prec_gen;
}

// V = Q_R V_M (n x l row-major in Vhat) of the explicit P, formed once per
// build for the one-column P-apply (the blocked path does without it).
static void ensure_vhat(Ctx& c, hipStream_t s) {
  if (!c.have_prec || c.o.precond != 1 || c.prec.implicit) return;
  if (c.vhat_kind == 1 && c.vhat_gen == c.prec_gen) return;
  const int l = c.prec.ell;
  gemm(c, Op::T, Op::T, l, c.n, l, 1.0, c.Vm, c.vm_ld, c.Q, c.n, 0.0, c.Vhat, l);
  c.vhat_kind = 1;
  c.vhat_gen = c.prec_gen;
}

// ------------------------------------------------------------------ LSQR phases
struct PhaseOut {
  int iters;
  int reason;
};

static GKVecs<double> vecs(Ctx& c) { return GKVecs<double>{c.u_top, c.u_bot, c.v, c.w, c.y, c.t, c.g}; }

static void upload_state(Ctx& c, double tol_abs, double pnorm, double eps_lsqr, double baug_eps, double nu,
                         double sigma_l, int max_iter, double delta, hipStream_t s, double rel_tol = 0.0) {
  GKState& h = c.st_host[0];
  std::memset(&h, 0, sizeof(h));
  h.rel_tol = rel_tol;
  h.alpha = 1.0;
  h.beta = 1.0;
  h.pnorm = pnorm;
  h.tol_abs = tol_abs;
  h.eps_lsqr = eps_lsqr;
  h.baug_eps = baug_eps;
  h.nu = nu;
  h.sigma_l = sigma_l;
  h.delta = delta;
  h.max_iter = max_iter;
  h.init = 1;
  set_state(c.st, h, s);
}

// Both slots; the returned state is slot 0 unless only slot 1 carries the
// stop flag (a stop found while finishing beta).
static GKState read_state(Ctx& c, hipStream_t s) {
  APL_HIP(hipMemcpyAsync(c.st_host, c.st, 2 * sizeof(GKState), hipMemcpyDeviceToHost, s));
  APL_HIP(hipStreamSynchronize(s));
  if (c.st_host[1].stop && !c.st_host[0].stop) return c.st_host[1];
  return c.st_host[0];
}

// Relative reduction of the preconditioned normal residual that ends an FP32
// phase: below it the FP32 recurrences stop converging, and the next phase
// restarts from the FP64 residual (iterative refinement).
constexpr double kFp32PhaseRelTol = 1e-5;
// BF16 blocked products (precision 2): a phase stops at 1e-2 of its starting
// normal residual (about the relative rounding of the BF16 values), and BF16
// stays in use while every phase divides eta by at least 1 / kBf16MinGain.
constexpr double kBf16PhaseRelTol = 1e-2;
constexpr double kBf16MinGain = 0.1;

// Iterations per captured graph (graphs option).
constexpr int kGraphChunk = 16;

// The captured chunk of kGraphChunk iterations for this operator / P /
// precision, captured again when any of them changes.  Capture needs a
// stream other than the legacy default stream; returns null there.
template <class V>
static hipGraphExec_t phase_graph(Ctx& c, const OpDesc& A, GKVecs<V> vec, const PrecDesc* P, hipStream_t s) {
  if (s == nullptr) return nullptr;
  const long long key = (long long)sizeof(V) * 1000000007LL + (P ? 1 + 2LL * P->ell + (P->implicit ? 1 : 0) : 0) +
                        (A.f64 ? 0 : 500000000LL);
  if (c.gexec && c.gkey == key) return c.gexec;
  if (c.gexec) {
    SyncGuard gd(g_capture_mu);
    APL_HIP(hipGraphExecDestroy(c.gexec));
    c.gexec = nullptr;
  }
  hipGraph_t g = nullptr;
  std::unique_lock<std::shared_mutex> excl(g_capture_mu);
  APL_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  for (int i = 0; i < kGraphChunk; ++i) gk_iteration<V>(A, P, vec, c.st, c.wk, s);
  const hipError_t e1 = hipGetLastError();
  const hipError_t e2 = hipStreamEndCapture(s, &g);
  if (e1 != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    throw Error(APLICUR_E_HIP, std::string("graph capture failed: ") + hipGetErrorString(e1 != hipSuccess ? e1 : e2));
  }
  excl.unlock();
  SyncGuard gi(g_capture_mu);
  hipGraphExec_t ex = nullptr;
  const hipError_t e3 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e3 != hipSuccess) throw Error(APLICUR_E_HIP, std::string("graph instantiation failed: ") + hipGetErrorString(e3));
  c.gexec = ex;
  c.gkey = key;
  return ex;
}

template <class V>
static PhaseOut run_phase_t(Ctx& c, const OpDesc& A, GKVecs<V> vec, const PrecDesc* P, const double* b,
                            const double* b_bot, double bot_scale, double* x, bool x_zero, hipStream_t s) {
  gk_phase_init<V>(c.op, A, P, b, b_bot, bot_scale, x_zero ? nullptr : x, vec, c.st, c.wk, s);
  int chunk = 8;
  long long launched = 0;
  APL_HIP(hipGetLastError());
  hipGraphExec_t gx = c.o.graphs ? phase_graph<V>(c, A, vec, P, s) : nullptr;
  GKState h = read_state(c, s);
  const long long budget = h.max_iter;
  while (!h.stop) {
    if (gx) {
      APL_HIP(hipGraphLaunch(gx, s));
      launched += kGraphChunk;
    } else {
      for (int i = 0; i < chunk; ++i) gk_iteration<V>(A, P, vec, c.st, c.wk, s);
      launched += chunk;
      chunk = std::min(chunk * 2, 64);
    }
    APL_HIP(hipGetLastError());
    h = read_state(c, s);
    if (!h.stop && launched > budget + 128)
      throw Error(APLICUR_E_HIP, "LSQR phase did not reach its stopping test within its budget");
  }
  if (h.reason == 6) throw Error(APLICUR_E_BREAKDOWN, "non-finite value in the LSQR recurrence");
  gk_phase_finish<V>(A, P, vec, x, c.st, s);
  return PhaseOut{h.iter, h.reason};
}

// One warm-started phase for the problem min || A_mu x - [b; bot_scale b_bot] ||
// (FP64, or FP32 recurrences from an FP64 residual with precision 1).
static PhaseOut run_phase(Ctx& c, const PrecDesc* P, const double* b, const double* b_bot, double bot_scale,
                          double* x, bool x_zero, double tol_abs, double pnorm, double eps_lsqr, double baug_eps,
                          double nu, double sigma_l, int budget, hipStream_t s) {
  const GKVecs<float> v32{c.u_top32, c.u_bot32, c.v32, c.w32, c.y32, c.t32, c.g32};
  const bool refinement = std::isinf(nu) && eps_lsqr == 0.0;  // final / refinement phases
  if (c.fp32 && (x_zero || !refinement || c.delta > 0.0)) {
    if (!x_zero && refinement) {
      // FP32 refinement phase: the correction d = (A^T A + mu I)^{-1} s with
      // s = A_mu^T r (FP64) solves min || A_mu d - [0; s / delta] ||, whose
      // right-hand side shrinks with the normal residual (the residual r
      // itself stays at the least-squares residual, which FP32 cannot
      // resolve to the requested eta).  Intermediate phases (dynamic stop)
      // keep the warm-restart form of Sec. 3.2 below.
      upload_state(c, 0.0, 1.0, 0.0, 0.0, INFINITY, 0.0, 1, c.delta, s);
      gk_normal_vector(c.op, b, b_bot, bot_scale, x, c.u_top, c.u_bot, c.g, c.st, c.wk, s);
      upload_state(c, tol_abs, pnorm, eps_lsqr, baug_eps, nu, sigma_l, budget, c.delta, s, kFp32PhaseRelTol);
      return run_phase_t<float>(c, c.op32, v32, P, nullptr, c.g, 1.0 / c.delta, x, true, s);
    }
    upload_state(c, tol_abs, pnorm, eps_lsqr, baug_eps, nu, sigma_l, budget, c.delta, s, kFp32PhaseRelTol);
    return run_phase_t<float>(c, c.op32, v32, P, b, b_bot, bot_scale, x, x_zero, s);
  }
  // FP64 phase (also the refinement phases of precision 1 when mu = 0)
  upload_state(c, tol_abs, pnorm, eps_lsqr, baug_eps, nu, sigma_l, budget, c.delta, s);
  return run_phase_t<double>(c, c.op, vecs(c), P, b, b_bot, bot_scale, x, x_zero, s);
}

// eta = ||A_mu^T r|| / atb with r the residual of x, FP64 from scratch.
static double eta_of(Ctx& c, const double* b, const double* b_bot, double bot_scale, const double* x, double atb,
                     hipStream_t s) {
  if (atb == 0.0) return 0.0;
  upload_state(c, 0.0, 1.0, 0.0, 0.0, INFINITY, 0.0, 1, c.delta, s);
  gk_normal_residual(c.op, b, b_bot, bot_scale, x, vecs(c), c.st, c.wk, s);
  GKState h = read_state(c, s);
  return std::sqrt(std::max(h.h2, 0.0)) / atb;
}

static double atb_norm(Ctx& c, const double* b, hipStream_t s) {
  upload_state(c, 0.0, 1.0, 0.0, 0.0, INFINITY, 0.0, 1, 0.0, s);
  op_atb_norm2(c.op, b, c.g, c.st, c.wk, s);
  GKState h = read_state(c, s);
  return std::sqrt(std::max(h.h2, 0.0));
}

static double vec_norm(Ctx& c, const double* b, hipStream_t s) {
  upload_state(c, 0.0, 1.0, 0.0, 0.0, INFINITY, 0.0, 1, 0.0, s);
  op_norm(c.op, b, nullptr, 0.0, c.u_top, c.u_bot, c.st, c.wk, s);
  GKState h = read_state(c, s);
  return h.beta;
}

// ||g|| of an n-vector (the bottom block of [0; g], delta = 1).
static double vec_norm_n(Ctx& c, const double* g, hipStream_t s) {
  upload_state(c, 0.0, 1.0, 0.0, 0.0, INFINITY, 0.0, 1, 1.0, s);
  op_norm(c.op, nullptr, g, 1.0, c.u_top, c.u_bot, c.st, c.wk, s);
  GKState h = read_state(c, s);
  return h.beta;
}

struct ColState {
  double atb = 0.0, bnorm = 0.0, eta = INFINITY;
  int used = 0, phases = 0;
  bool done = false;
};

// Right-hand side of one column: [b; bot_scale b_bot] (b or b_bot may be null).
struct Rhs {
  const double* b;
  const double* b_bot;
  double bot_scale;
};

// Solve one column with P fixed (plain LSQR when P is null): restarted phases
// with nu = inf until eta <= tol or the budget/stall guard ends it.
static void refine(Ctx& c, const PrecDesc* P, Rhs r, double* x, ColState& cs, double pnorm, double sigma_l,
                   bool first_from_zero, std::vector<int>* it_log, std::vector<double>* eta_log, hipStream_t s) {
  int stalls = 0;
  bool xz = first_from_zero;
  while (cs.eta > c.o.tol_ne && cs.used < c.o.max_iter && stalls < 3) {
    const double prev = cs.eta;
    PhaseOut po = run_phase(c, P, r.b, r.b_bot, r.bot_scale, x, xz, c.o.tol_ne * cs.atb, pnorm, 0.0, 0.0, INFINITY,
                            sigma_l, c.o.max_iter - cs.used, s);
    xz = false;
    cs.used += po.iters;
    cs.phases += 1;
    cs.eta = eta_of(c, r.b, r.b_bot, r.bot_scale, x, cs.atb, s);
    if (it_log) it_log->push_back(po.iters);
    if (eta_log) eta_log->push_back(cs.eta);
    if (po.iters == 0 || po.reason == kStopBudget) break;
    stalls = (cs.eta > 0.5 * prev) ? stalls + 1 : 0;
  }
}

// Times and counters of one solve.
struct SolveLog {
  double t_cur = 0.0, t_prec = 0.0, t_lsqr = 0.0, last_rho = 0.0;
  int rebuilds = 0, outer = 0;
};

// The outer loop of Alg. 3 (CUR increments, the re-preconditioning test and
// P rebuilds).  After each rebuild, phases(final_step, nu, eps_lsqr) runs the
// LSQR work of the columns still active and returns whether any remains.
template <class Phases>
static void outer_loop(Ctx& c, hipStream_t s, SolveLog& lg, Phases&& phases) {
  // restart the CUR sequence (it depends on A only)
  c.rank = 0;
  c.I.clear();
  c.J.clear();
  c.rho_hist.clear();
  c.rank_hist.clear();
  c.rebuild_hist.clear();
  c.sweep_hist.clear();
  c.have_prec = false;
  c.vm_rank = 0;
  APL_HIP(hipMemcpyAsync(c.E, c.Y, sizeof(double) * (size_t)c.s * c.n, hipMemcpyDeviceToDevice, s));
  double d_cur = INFINITY;
  for (;;) {
    auto t0 = Clock::now();
    StepResult sr = outer_step(c, s);
    lg.t_cur += ms_since(t0);
    ++lg.outer;
    if (sr.added == 0 && c.rank == 0) break;
    lg.last_rho = sr.rho;
    // schedule 0: Alg. 3; 1 / 2: single shot, P built once at the final rank
    // (2: the rank cap regardless of rho)
    const bool grown = sr.exhausted || c.rank >= c.L || (c.o.max_outer > 0 && lg.outer >= c.o.max_outer);
    const bool final_step = grown || (c.o.schedule != 2 && sr.rho <= c.eps_cur);
    const double gap = sr.rho - c.eps_cur;
    const bool rebuild = final_step || (c.o.schedule == 0 && d_cur / gap >= c.o.nu_prec);
    c.rho_hist.push_back(sr.rho);
    c.rank_hist.push_back(c.rank);
    c.rebuild_hist.push_back(rebuild ? 1 : 0);
    bool any_active = true;
    if (rebuild) {
      t0 = Clock::now();
      build_precond(c, s);
      ++lg.rebuilds;
      lg.t_prec += ms_since(t0);
      t0 = Clock::now();
      any_active = phases(final_step, final_step ? INFINITY : c.o.nu_lsqr, final_step ? 0.0 : c.o.eps_lsqr);
      d_cur = gap;
      lg.t_lsqr += ms_since(t0);
    }
    if (final_step || !any_active) break;
  }
}

static void fill_info(Ctx& c, const std::vector<ColState>& cols, const SolveLog& lg, aplicur_info* info, int& status) {
  status = APLICUR_OK;
  double eta_max = 0.0;
  int iters = 0, phases = 0;
  for (auto& cs : cols) {
    eta_max = std::max(eta_max, cs.eta);
    iters = std::max(iters, cs.used);
    phases = std::max(phases, cs.phases);
    if (cs.eta > c.o.tol_ne) status = APLICUR_W_MAXITER;
  }
  if (info) {
    info->status = status;
    info->phases = phases;
    info->iters = iters;
    info->rank = c.rank;
    info->rebuilds = lg.rebuilds;
    info->outer = lg.outer;
    info->eta = eta_max;
    info->rho = lg.last_rho;
    info->sigma_hat = c.p_target;
    info->t_sketch_ms = c.t_sketch;
    info->t_cur_ms = lg.t_cur;
    info->t_precond_ms = lg.t_prec;
    info->t_lsqr_ms = lg.t_lsqr;
  }
}

static bool use_blocked(const Ctx& c, int nrhs);
static int solve_blocked(Ctx& c, const double* B, long long ldb, int nrhs, double* X, long long ldx, bool warm,
                         aplicur_info* info, hipStream_t s);

static int solve(Ctx& c, const double* B, long long ldb, int nrhs, double* X, long long ldx, bool warm,
                 aplicur_info* info, hipStream_t s) {
  APL_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
  APL_REQUIRE(B && X, "null B or X");
  APL_REQUIRE(ldb >= c.m && ldx >= c.n, "ldb must be >= m and ldx >= n");
  set_stream(c, s);
  if (use_blocked(c, nrhs)) return solve_blocked(c, B, ldb, nrhs, X, ldx, warm, info, s);
  std::vector<ColState> cols(nrhs);
  for (int k = 0; k < nrhs; ++k) {
    const double* b = B + (size_t)k * ldb;
    double* x = X + (size_t)k * ldx;
    if (!warm) fill(x, c.n, 0.0, s);
    cols[k].atb = atb_norm(c, b, s);
    cols[k].bnorm = vec_norm(c, b, s);
    if (!std::isfinite(cols[k].atb) || !std::isfinite(cols[k].bnorm))
      throw Error(APLICUR_E_BREAKDOWN, "non-finite values in A or B");
    if (cols[k].atb == 0.0) {
      fill(x, c.n, 0.0, s);
      cols[k].eta = 0.0;
      cols[k].done = true;
    } else if (warm) {
      cols[k].eta = eta_of(c, b, nullptr, 0.0, x, cols[k].atb, s);
      cols[k].done = cols[k].eta <= c.o.tol_ne;
    }
  }
  c.phase_iters0.clear();
  c.phase_eta0.clear();
  SolveLog lg;
  bool any_active = false;
  for (auto& cs : cols) any_active |= !cs.done;
  if (!c.o.precond) {
    auto t0 = Clock::now();
    for (int k = 0; k < nrhs; ++k) {
      if (cols[k].done) continue;
      refine(c, nullptr, Rhs{B + (size_t)k * ldb, nullptr, 0.0}, X + (size_t)k * ldx, cols[k], 1.0, 0.0, !warm,
             k == 0 ? &c.phase_iters0 : nullptr, k == 0 ? &c.phase_eta0 : nullptr, s);
      cols[k].done = true;
    }
    lg.t_lsqr += ms_since(t0);
  } else if (any_active) {
    outer_loop(c, s, lg, [&](bool final_step, double nu, double epsl) {
      ensure_vhat(c, s);
      bool active = false;
      for (int k = 0; k < nrhs; ++k) {
        ColState& cs = cols[k];
        if (cs.done) continue;
        const double* b = B + (size_t)k * ldb;
        double* x = X + (size_t)k * ldx;
        const bool xz = (!warm && cs.phases == 0);
        PhaseOut po = run_phase(c, &c.prec, b, nullptr, 0.0, x, xz, c.o.tol_ne * cs.atb, c.p_pnorm, epsl,
                                c.o.eps_lsqr * cs.bnorm, nu, c.p_sigma_l, c.o.max_iter - cs.used, s);
        cs.used += po.iters;
        cs.phases += 1;
        cs.eta = eta_of(c, b, nullptr, 0.0, x, cs.atb, s);
        if (k == 0) {
          c.phase_iters0.push_back(po.iters);
          c.phase_eta0.push_back(cs.eta);
        }
        if (cs.eta <= c.o.tol_ne || cs.used >= c.o.max_iter) {
          cs.done = true;
        } else if (final_step) {
          refine(c, &c.prec, Rhs{b, nullptr, 0.0}, x, cs, c.p_pnorm, c.p_sigma_l, false,
                 k == 0 ? &c.phase_iters0 : nullptr, k == 0 ? &c.phase_eta0 : nullptr, s);
          cs.done = true;
        }
        active |= !cs.done;
      }
      return active;
    });
  }
  int status = APLICUR_OK;
  fill_info(c, cols, lg, info, status);
  return status;
}

// ------------------------------------------------------------------ blocked path
// Several right-hand sides of a dense A: groups of up to 64 columns run their
// LSQR recurrences together, the products as MFMA matrix products (A read
// once per iteration for the whole group instead of once per column).  Same
// phases, stopping tests and refinement as the column path, per column.
constexpr int kBlkMaxCols = 64;

static bool use_blocked(const Ctx& c, int nrhs) {
  // the blocked P-apply has the SVD form's diagonal middle factor only
  return nrhs >= 2 && !c.op.csr && !c.o.columns && c.o.precond != 2;
}

static int blk_kp(int k) { return k <= 16 ? 16 : (k <= 32 ? 32 : 64); }

static void ensure_blk(Ctx& c, int kp, hipStream_t s) {
  if (!c.blk) c.blk = std::make_unique<Blk>();
  Blk& b = *c.blk;
  b.nres.ok = false;  // every caller goes on to write Bp, Xp, tm / tn or the planes
  const long long m = c.m, n = c.n;
  const size_t vs = c.op.f64 ? 8 : 4;
  if (!b.At) {
    b.ldt = (m + 3) / 4 * 4;
    b.At = c.arena.alloc<char>(vs * (size_t)n * b.ldt);
    if (c.op.f64)
      transpose_rect<double>((const double*)c.op.val, m, n, c.op.ld, (double*)b.At, b.ldt, s);
    else
      transpose_rect<float>((const float*)c.op.val, m, n, c.op.ld, (float*)b.At, b.ldt, s);
    b.op.A = c.op.val;
    b.op.At = b.At;
    b.op.m = m;
    b.op.n = n;
    b.op.ld = c.op.ld;
    b.op.ldt = b.ldt;
    b.op.f64 = c.op.f64;
    b.op.Sm = gemm_splits(m, n);
    b.op.Sn = gemm_splits(n, m);
    if (c.o.precond) b.W = c.arena.alloc<double>((size_t)std::max(c.L, 1) * std::max(c.L, 1));
  }
  if (c.fp32 && !b.op32.A) {
    b.op32 = b.op;
    b.op32.f64 = 0;
    b.op32.A = c.op32.val;
    b.op32.ld = c.op32.ld;
    if (c.op.f64) {
      b.At32 = c.arena.alloc<float>((size_t)n * b.ldt);
      transpose_rect<float>((const float*)c.op32.val, m, n, c.op32.ld, (float*)b.At32, b.ldt, s);
      b.op32.At = b.At32;
    }
  }
  if (c.bf16 && !b.A16) {
    b.A16 = c.arena.alloc<uint16_t>((size_t)bf16_tiled_elems(m, n));
    b.At16 = c.arena.alloc<uint16_t>((size_t)bf16_tiled_elems(n, m));
    tile_bf16((const float*)b.op32.A, m, n, b.op32.ld, b.A16, s);
    tile_bf16((const float*)b.op32.At, n, m, b.op32.ldt, b.At16, s);
    b.op16 = b.op32;
    b.op16.A16 = b.A16;
    b.op16.At16 = b.At16;
  }
  if (b.kp >= kp) return;
  b.kp = kp;
  if (c.fp32) {
    b.vec32.u_top = c.arena.alloc<float>((size_t)m * kp);
    b.vec32.u_bot = c.arena.alloc<float>((size_t)n * kp);
    b.vec32.v = c.arena.alloc<float>((size_t)n * kp);
    b.vec32.w = c.arena.alloc<float>((size_t)n * kp);
    b.vec32.y = c.arena.alloc<float>((size_t)n * kp);
    b.vec32.t = c.arena.alloc<float>((size_t)n * kp);
    b.vec32.g = c.arena.alloc<float>((size_t)n * kp);
    b.Nc = c.arena.alloc<double>((size_t)n * kp);
  }
  const int L = std::max(c.L, 1);
  b.S1max = 64;
  b.S2max = gemm_splits(n, L);
  b.Bp = c.arena.alloc<double>((size_t)m * kp);
  b.Bbot = c.arena.alloc<double>((size_t)n * kp);
  b.Xp = c.arena.alloc<double>((size_t)n * kp);
  b.tm = c.arena.alloc<double>((size_t)m * kp);
  b.tn = c.arena.alloc<double>((size_t)n * kp);
  b.vec.u_top = c.arena.alloc<double>((size_t)m * kp);
  b.vec.u_bot = c.arena.alloc<double>((size_t)n * kp);
  b.vec.v = c.arena.alloc<double>((size_t)n * kp);
  b.vec.w = c.arena.alloc<double>((size_t)n * kp);
  b.vec.y = c.arena.alloc<double>((size_t)n * kp);
  b.vec.t = c.arena.alloc<double>((size_t)n * kp);
  b.vec.g = c.arena.alloc<double>((size_t)n * kp);
  b.wk.pm = c.arena.alloc<double>((size_t)b.op.Sm * m * kp);
  b.wk.pn = c.arena.alloc<double>((size_t)b.op.Sn * n * kp);
  if (c.o.precond) {
    b.wk.pl = c.arena.alloc<double>((size_t)b.S1max * L * kp);
    b.wk.pc = c.arena.alloc<double>((size_t)L * kp);
    b.wk.pc2 = c.arena.alloc<double>((size_t)L * kp);
    b.wk.pq = c.arena.alloc<double>((size_t)b.S2max * n * kp);
  }
  b.wk.beta_part = c.arena.alloc<double>((size_t)kBlkMaxGrid * kp);
  b.wk.alpha_part = c.arena.alloc<double>((size_t)kBlkMaxGrid * kp);
  b.wk.norm_part = c.arena.alloc<double>((size_t)kBlkMaxGrid * kp);
  b.st = c.arena.alloc<GKState>(2 * kp);
  SyncGuard g(g_capture_mu);
  if (b.st_up) (void)hipHostFree(b.st_up);
  if (b.st_down) (void)hipHostFree(b.st_down);
  if (b.norm_host) (void)hipHostFree(b.norm_host);
  b.st_up = b.st_down = nullptr;
  b.norm_host = nullptr;
  APL_HIP(hipHostMalloc((void**)&b.st_up, sizeof(GKState) * 2 * kp, hipHostMallocDefault));
  APL_HIP(hipHostMalloc((void**)&b.st_down, sizeof(GKState) * 2 * kp, hipHostMallocDefault));
  APL_HIP(hipHostMalloc((void**)&b.norm_host, sizeof(double) * kBlkMaxGrid * kp, hipHostMallocDefault));
}

// The explicit P for the blocked kernels in factored form: V = Q_R V_M, so
// V diag(d) V^T = Q_R W Q_R^T with W = V_M diag(d) V_M^T (ell x ell,
// symmetric; an ell^3 product per build instead of the n ell^2 one that
// forms V).  Q_R^T z is a product with Q itself (column-major n x l =
// row-major l x n), then W, then Q_R (its row-major copy in Vhat).  W and
// the copy are refreshed after each rebuild.
static BlkPrec blk_prec(Ctx& c, hipStream_t s) {
  Blk& b = *c.blk;
  const int l = c.prec.ell, lp = c.vm_ld;
  APL_REQUIRE(b.W, "blocked P buffers missing");
  if (c.vhat_kind != 2 || c.vhat_gen != c.prec_gen) {
    transpose_rect<double>(c.Q, l, c.n, c.n, c.Vhat, l, s);  // Q_R row-major, n x l
    c.vhat_kind = 2;
    c.vhat_gen = c.prec_gen;
  }
  if (b.w_gen != c.prec_gen) {
    copy_block(c.Vm, lp, c.Kc, l, l, l, 1.0, s);  // V_M (ld l)
    scale_cols(c.Kc, l, l, l, c.d, c.Kr, s);       // V_M diag(d)
    gemm(c, Op::N, Op::T, l, l, l, 1.0, c.Kr, l, c.Kc, l, 0.0, b.W, l);
    b.w_gen = c.prec_gen;
  }
  BlkPrec P{};
  P.V = c.Vhat;
  P.ldv = l;
  P.Vt = c.Q;
  P.ldvt = c.n;
  P.W = b.W;
  P.d = c.prec.d;
  P.ell = l;
  P.S1 = std::min(b.S1max, gemm_splits(l, c.n));
  P.S2 = std::min(b.S2max, gemm_splits(c.n, l));
  P.S3 = std::min(b.S1max, gemm_splits(l, l));
  return P;
}

// Per-column norms (sqrt of the column sums of the norm partials).
static std::vector<double> blk_col_norms(Ctx& c, int k, int mode, const double* B, const double* Bbot, double bs,
                                         const double* X, hipStream_t s) {
  Blk& b = *c.blk;
  const int kp = b.kp;
  const int cnt = blk_norms(b.op, kp, mode, B, Bbot, bs, X, c.delta, b.tm, b.tn, b.wk, s);
  if (mode == 1 || mode == 2) {
    b.nres.ok = B == b.Bp && (mode == 1 || X == b.Xp);
    b.nres.x_zero = mode == 1;
    b.nres.Bbot = Bbot;
    b.nres.bs = bs;
  }
  APL_HIP(hipMemcpyAsync(b.norm_host, b.wk.norm_part, sizeof(double) * cnt * kp, hipMemcpyDeviceToHost, s));
  APL_HIP(hipStreamSynchronize(s));
  std::vector<double> out(k, 0.0);
  for (int j = 0; j < k; ++j) {
    double t = 0.0;
    for (int w = 0; w < cnt; ++w) t += b.norm_host[(size_t)w * kp + j];
    out[j] = std::sqrt(std::max(t, 0.0));
  }
  return out;
}

// Stopping parameters of one column for one phase (inactive: starts stopped).
struct BlkParam {
  bool active = false;
  double tol_abs = 0.0, pnorm = 1.0, eps_lsqr = 0.0, baug_eps = 0.0, nu = INFINITY, sigma_l = 0.0;
  int budget = 0;
};

// Work per queued chunk of blocked iterations (seconds at an assumed stream
// rate of the products).
constexpr double kBlkChunkSeconds = 1.0e-3;
constexpr double kBlkChunkBytesPerSecond = 4.0e12;

// One warm-started phase for the active columns of min || A_mu X - [B; bs Bbot] ||:
// FP64, or with precision 1 FP32 recurrences from an FP64 residual; FP32
// refinement phases (nu = inf, eps_lsqr = 0, X warm, delta > 0) solve for the
// correction with the right-hand side [0; A_mu^T r / delta], as the column path.
template <class V>
static std::vector<PhaseOut> run_phase_blk_t(Ctx& c, const BlkOp& A, BlkVecs<V> vec, const BlkPrec* P,
                                             const std::vector<BlkParam>& prm, const double* B, const double* Bbot,
                                             double bs, bool x_zero, double rel_tol, hipStream_t s,
                                             const double* r_ready = nullptr) {
  Blk& b = *c.blk;
  const int kp = b.kp, k = (int)prm.size();
  long long budget = 0;
  for (int j = 0; j < kp; ++j) {
    GKState& h = b.st_up[j];
    std::memset(&h, 0, sizeof(h));
    h.alpha = 1.0;
    h.beta = 1.0;
    h.delta = c.delta;
    h.rel_tol = rel_tol;
    if (j < k && prm[j].active) {
      const BlkParam& q = prm[j];
      h.pnorm = q.pnorm;
      h.tol_abs = q.tol_abs;
      h.eps_lsqr = q.eps_lsqr;
      h.baug_eps = q.baug_eps;
      h.nu = q.nu;
      h.sigma_l = q.sigma_l;
      h.max_iter = q.budget;
      h.init = 1;
      budget = std::max<long long>(budget, q.budget);
    } else {
      h.stop = 1;
      h.nu = INFINITY;
    }
    b.st_up[kp + j] = h;
  }
  APL_HIP(hipMemcpyAsync(b.st, b.st_up, sizeof(GKState) * 2 * kp, hipMemcpyHostToDevice, s));
  blk_phase_init<V>(b.op, A, P, kp, B, Bbot, bs, b.Xp, x_zero, c.delta, vec, b.st, b.wk, s, r_ready);
  auto read = [&]() {
    APL_HIP(hipMemcpyAsync(b.st_down, b.st, sizeof(GKState) * 2 * kp, hipMemcpyDeviceToHost, s));
    APL_HIP(hipStreamSynchronize(s));
    bool all = true;
    for (int j = 0; j < k; ++j) {
      if (!prm[j].active) continue;
      const GKState& h0 = b.st_down[j];
      const GKState& h1 = b.st_down[kp + j];
      all &= (h0.stop || h1.stop);
    }
    return all;
  };
  // Iterations are queued in chunks between reads of the stop flags.  The
  // blocked products do their whole work even after every column has stopped,
  // so the chunk is capped to about kBlkChunkSeconds of estimated work: one
  // iteration per read when an iteration streams gigabytes (the wait for the
  // read is then a small fraction of it), up to 64 when it is short.
  const double elem = A.A16 ? 2.0 : (A.f64 ? 8.0 : 4.0);
  double iter_bytes = 2.0 * (double)A.m * (double)A.n * elem;
  if (P) iter_bytes += 4.0 * (double)A.n * (double)P->ell * 8.0;
  const int cap = (int)std::max(1.0, std::min(64.0, kBlkChunkSeconds * kBlkChunkBytesPerSecond / iter_bytes));
  int chunk = std::min(8, cap);
  long long launched = 0;
  APL_HIP(hipGetLastError());
  bool done = read();
  while (!done) {
    for (int i = 0; i < chunk; ++i) blk_iteration<V>(A, P, kp, c.delta, vec, b.st, b.wk, s);
    launched += chunk;
    chunk = std::min(chunk * 2, cap);
    APL_HIP(hipGetLastError());
    done = read();
    if (!done && launched > budget + 128)
      throw Error(APLICUR_E_HIP, "blocked LSQR phase did not reach its stopping tests within its budget");
  }
  std::vector<PhaseOut> out(k, PhaseOut{0, kStopNone});
  for (int j = 0; j < k; ++j) {
    if (!prm[j].active) continue;
    const GKState& h0 = b.st_down[j];
    const GKState& h1 = b.st_down[kp + j];
    const GKState& h = (h1.stop && !h0.stop) ? h1 : h0;
    if (h.reason == 6) throw Error(APLICUR_E_BREAKDOWN, "non-finite value in the LSQR recurrence");
    out[j] = PhaseOut{h.iter, h.reason};
  }
  blk_phase_finish<V>(A, P, kp, vec, b.Xp, b.wk, s);
  return out;
}

static std::vector<PhaseOut> run_phase_blk(Ctx& c, const BlkPrec* P, const std::vector<BlkParam>& prm,
                                           const double* Bbot, double bs, bool x_zero, hipStream_t s) {
  Blk& b = *c.blk;
  bool refinement = true;
  for (const BlkParam& q : prm)
    if (q.active) refinement &= std::isinf(q.nu) && q.eps_lsqr == 0.0;
  b.last_bf16 = false;
  const bool reuse = b.nres.ok && b.nres.x_zero == x_zero && b.nres.Bbot == Bbot && b.nres.bs == bs;
  b.nres.ok = false;
  if (c.fp32 && (x_zero || !refinement || c.delta > 0.0)) {
    const bool use16 = c.bf16 && b.bf16_live;
    const BlkOp& op = use16 ? b.op16 : b.op32;
    const double rt = use16 ? kBf16PhaseRelTol : kFp32PhaseRelTol;
    b.last_bf16 = use16;
    b.phases16 += use16 ? 1 : 0;
    if (!x_zero && refinement) {
      // N = A_mu^T r (FP64) of the current X, then the correction from zero
      (void)blk_norms(b.op, b.kp, 2, b.Bp, Bbot, bs, b.Xp, c.delta, b.tm, b.tn, b.wk, s, b.Nc);
      return run_phase_blk_t<float>(c, op, b.vec32, P, prm, nullptr, b.Nc, 1.0 / c.delta, true, rt, s);
    }
    return run_phase_blk_t<float>(c, op, b.vec32, P, prm, b.Bp, Bbot, bs, x_zero, rt, s);
  }
  const double* r_ready = reuse ? (x_zero ? b.Bp : b.tm) : nullptr;
  return run_phase_blk_t<double>(c, b.op, b.vec, P, prm, b.Bp, Bbot, bs, x_zero, 0.0, s, r_ready);
}

// After a phase with BF16 products: if some column's eta fell by less than
// kBf16MinGain, the rest of the solve takes the FP32 products.
static void bf16_ladder(Ctx& c, const std::vector<BlkParam>& prm, const std::vector<double>& before,
                        const std::vector<ColState>& cols) {
  Blk& b = *c.blk;
  if (!b.last_bf16) return;
  for (size_t j = 0; j < prm.size(); ++j)
    if (prm[j].active && cols[j].eta > kBf16MinGain * before[j]) b.bf16_live = false;
}

// Restarted phases with nu = inf for every column not yet done, until each
// reaches eta <= tol or its budget / stall guard (the column path's refine).
static void refine_blk(Ctx& c, const BlkPrec* P, std::vector<ColState>& cols, const double* Bbot, double bs,
                       double pnorm, double sigma_l, bool first_from_zero, hipStream_t s) {
  const int k = (int)cols.size();
  std::vector<int> stalls(k, 0);
  std::vector<bool> live(k);
  for (int j = 0; j < k; ++j) live[j] = !cols[j].done;
  bool xz = first_from_zero;
  for (;;) {
    std::vector<BlkParam> prm(k);
    bool any = false;
    for (int j = 0; j < k; ++j) {
      ColState& cs = cols[j];
      if (live[j] && !(cs.eta > c.o.tol_ne && cs.used < c.o.max_iter && stalls[j] < 3)) live[j] = false;
      if (!live[j]) continue;
      BlkParam& q = prm[j];
      q.active = true;
      q.tol_abs = c.o.tol_ne * cs.atb;
      q.pnorm = pnorm;
      q.sigma_l = sigma_l;
      q.budget = c.o.max_iter - cs.used;
      any = true;
    }
    if (!any) break;
    std::vector<double> prev(k);
    for (int j = 0; j < k; ++j) prev[j] = cols[j].eta;
    std::vector<PhaseOut> po = run_phase_blk(c, P, prm, Bbot, bs, xz, s);
    xz = false;
    std::vector<double> eta = blk_col_norms(c, k, 2, c.blk->Bp, Bbot, bs, c.blk->Xp, s);
    for (int j = 0; j < k; ++j) {
      if (!prm[j].active) continue;
      ColState& cs = cols[j];
      cs.used += po[j].iters;
      cs.phases += 1;
      cs.eta = eta[j] / cs.atb;
      if (po[j].iters == 0 || po[j].reason == kStopBudget) live[j] = false;
      stalls[j] = (cs.eta > 0.5 * prev[j]) ? stalls[j] + 1 : 0;
    }
    bf16_ladder(c, prm, prev, cols);
  }
  for (auto& cs : cols) cs.done = true;
}

static int solve_blocked(Ctx& c, const double* B, long long ldb, int nrhs, double* X, long long ldx, bool warm,
                         aplicur_info* info, hipStream_t s) {
  std::vector<ColState> all(nrhs);
  SolveLog lg;
  c.phase_iters0.clear();
  c.phase_eta0.clear();
  for (int g0 = 0; g0 < nrhs; g0 += kBlkMaxCols) {
    const int k = std::min(kBlkMaxCols, nrhs - g0);
    const int kp = blk_kp(k);
    ensure_blk(c, kp, s);
    Blk& b = *c.blk;
    b.bf16_live = c.bf16;
    if (g0 == 0) b.phases16 = 0;
    pack_cols(B + (size_t)g0 * ldb, ldb, c.m, k, b.Bp, b.kp, s);
    if (warm)
      pack_cols(X + (size_t)g0 * ldx, ldx, c.n, k, b.Xp, b.kp, s);
    else
      fill(b.Xp, c.n * b.kp, 0.0, s);
    std::vector<ColState> cols(k);
    const std::vector<double> atb = blk_col_norms(c, k, 1, b.Bp, nullptr, 0.0, nullptr, s);
    const std::vector<double> bn = blk_col_norms(c, k, 0, b.Bp, nullptr, 0.0, nullptr, s);
    std::vector<double> eta0;
    if (warm) eta0 = blk_col_norms(c, k, 2, b.Bp, nullptr, 0.0, b.Xp, s);
    for (int j = 0; j < k; ++j) {
      ColState& cs = cols[j];
      cs.atb = atb[j];
      cs.bnorm = bn[j];
      if (!std::isfinite(cs.atb) || !std::isfinite(cs.bnorm))
        throw Error(APLICUR_E_BREAKDOWN, "non-finite values in A or B");
      if (cs.atb == 0.0) {
        cs.eta = 0.0;
        cs.done = true;
      } else if (warm) {
        cs.eta = eta0[j] / cs.atb;
        cs.done = cs.eta <= c.o.tol_ne;
      }
    }
    bool any_active = false;
    for (auto& cs : cols) any_active |= !cs.done;
    SolveLog gl;
    if (!c.o.precond) {
      auto t0 = Clock::now();
      refine_blk(c, nullptr, cols, nullptr, 0.0, 1.0, 0.0, !warm, s);
      gl.t_lsqr += ms_since(t0);
    } else if (any_active) {
      outer_loop(c, s, gl, [&](bool final_step, double nu, double epsl) {
        const BlkPrec P = blk_prec(c, s);
        std::vector<BlkParam> prm(k);
        bool xz = !warm;
        for (int j = 0; j < k; ++j) {
          ColState& cs = cols[j];
          if (cs.done) continue;
          xz &= (cs.phases == 0);
          BlkParam& q = prm[j];
          q.active = true;
          q.tol_abs = c.o.tol_ne * cs.atb;
          q.pnorm = c.p_pnorm;
          q.eps_lsqr = epsl;
          q.baug_eps = c.o.eps_lsqr * cs.bnorm;
          q.nu = nu;
          q.sigma_l = c.p_sigma_l;
          q.budget = c.o.max_iter - cs.used;
        }
        std::vector<double> before(k);  // eta before the phase (1 at a cold start: X = 0)
        for (int j = 0; j < k; ++j) before[j] = (cols[j].phases == 0 && !warm) ? 1.0 : cols[j].eta;
        std::vector<PhaseOut> po = run_phase_blk(c, &P, prm, nullptr, 0.0, xz, s);
        const std::vector<double> eta = blk_col_norms(c, k, 2, c.blk->Bp, nullptr, 0.0, c.blk->Xp, s);
        bool rest = false;
        for (int j = 0; j < k; ++j) {
          if (!prm[j].active) continue;
          ColState& cs = cols[j];
          cs.used += po[j].iters;
          cs.phases += 1;
          cs.eta = eta[j] / cs.atb;
          if (cs.eta <= c.o.tol_ne || cs.used >= c.o.max_iter) cs.done = true;
          rest |= !cs.done;
        }
        bf16_ladder(c, prm, before, cols);
        if (final_step && rest) refine_blk(c, &P, cols, nullptr, 0.0, c.p_pnorm, c.p_sigma_l, false, s);
        bool active = false;
        for (auto& cs : cols) active |= !cs.done;
        return active;
      });
    }
    unpack_cols(b.Xp, b.kp, c.n, k, X + (size_t)g0 * ldx, ldx, s);
    for (int j = 0; j < k; ++j)
      if (cols[j].atb == 0.0) fill(X + (size_t)(g0 + j) * ldx, c.n, 0.0, s);
    for (int j = 0; j < k; ++j) all[g0 + j] = cols[j];
    lg.t_cur += gl.t_cur;
    lg.t_prec += gl.t_prec;
    lg.t_lsqr += gl.t_lsqr;
    lg.rebuilds += gl.rebuilds;
    lg.outer += gl.outer;
    lg.last_rho = gl.last_rho;
  }
  APL_HIP(hipStreamSynchronize(s));
  int status = APLICUR_OK;
  fill_info(c, all, lg, info, status);
  if (info) info->phases_bf16 = c.blk->phases16;
  return status;
}

// Y = A X (trans 0) or A^T X (trans 1) for k columns (column-major), in
// groups of up to 64 columns through the blocked products (dense A).
// prec 1 / 2: the FP32 / BF16 products of the low-precision phases.
// e0 / e1 (optional, k <= kBlkMaxCols): events on the product kernel's dispatch.
static void blk_apply(Ctx& c, int trans, const double* X, long long ldx, int k, double* Y, long long ldy,
                      hipStream_t s, int prec = 0, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  for (int g0 = 0; g0 < k; g0 += kBlkMaxCols) {
    const int kg = std::min(kBlkMaxCols, k - g0);
    ensure_blk(c, blk_kp(kg), s);
    Blk& b = *c.blk;
    void* part = trans ? b.wk.pn : b.wk.pm;
    if (prec == 0) {
      blk_matmat(b.op, trans != 0, X + (size_t)g0 * ldx, ldx, b.kp, kg, Y + (size_t)g0 * ldy, ldy, 0,
                 trans ? b.tm : b.tn, part, s, e0, e1);
    } else {
      float* in = trans ? b.vec32.u_top : b.vec32.t;
      blk_matmat(prec == 1 ? b.op32 : b.op16, trans != 0, X + (size_t)g0 * ldx, ldx, b.kp, kg,
                 Y + (size_t)g0 * ldy, ldy, prec, in, part, s, e0, e1);
    }
  }
}

// ------------------------------------------------------------------ adjoint
// Z = (A^T A + mu I)^{-1} G as min || A_mu Z - [0; G / delta] || by LSQR
// phases with the context's last preconditioner (plain LSQR if it has none),
// to eta_adj = ||G - (A^T A + mu I) Z|| / ||G|| <= tol_ne; then dB = A Z and
// dA = (B - A X) Z^T - (A Z) X^T (implicit differentiation of the normal
// equations; not part of the paper's method).
static int solve_backward(Ctx& c, const double* X, long long ldx, const double* B, long long ldb, const double* G,
                          long long ldg, int nrhs, double* Z, long long ldz, double* dB, long long lddb, double* dA,
                          long long ldda, aplicur_info* info, hipStream_t s) {
  APL_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
  APL_REQUIRE(c.delta > 0.0, "the adjoint needs mu > 0");
  APL_REQUIRE(G && Z && dB, "null G, Z or dB");
  APL_REQUIRE(ldg >= c.n && ldz >= c.n && lddb >= c.m, "leading dimensions too small");
  if (dA) {
    APL_REQUIRE(X && B, "dA needs X and B");
    APL_REQUIRE(ldx >= c.n && ldb >= c.m, "leading dimensions too small");
    APL_REQUIRE(c.op.csr || ldda >= (c.A.format == APLICUR_DENSE_COL ? c.m : c.n),
                "ldda must be >= n (row-major A) or >= m (column-major A)");
  }
  set_stream(c, s);
  auto t0 = Clock::now();
  const PrecDesc* P = c.have_prec ? &c.prec : nullptr;
  const double pnorm = c.have_prec ? c.p_pnorm : 1.0, sigma_l = c.have_prec ? c.p_sigma_l : 0.0;
  const bool blocked = use_blocked(c, nrhs);
  if (!blocked) ensure_vhat(c, s);
  int status = APLICUR_OK, iters = 0, phases = 0;
  double eta_max = 0.0;
  for (int g0 = 0; blocked && g0 < nrhs; g0 += kBlkMaxCols) {
    // the k columns of Z together (blocked path)
    const int kg = std::min(kBlkMaxCols, nrhs - g0);
    ensure_blk(c, blk_kp(kg), s);
    Blk& b = *c.blk;
    b.bf16_live = c.bf16;
    if (g0 == 0) b.phases16 = 0;
    BlkPrec Pb{};
    if (c.have_prec) Pb = blk_prec(c, s);
    fill(b.Bp, c.m * b.kp, 0.0, s);
    fill(b.Xp, c.n * b.kp, 0.0, s);
    pack_cols(G + (size_t)g0 * ldg, ldg, c.n, kg, b.Bbot, b.kp, s);
    const std::vector<double> gn = blk_col_norms(c, kg, 3, b.Bp, b.Bbot, 0.0, nullptr, s);
    std::vector<ColState> cols(kg);
    for (int j = 0; j < kg; ++j) {
      cols[j].atb = gn[j];
      if (!std::isfinite(gn[j])) throw Error(APLICUR_E_BREAKDOWN, "non-finite values in G");
      if (gn[j] == 0.0) {
        cols[j].eta = 0.0;
        cols[j].done = true;
      }
    }
    refine_blk(c, c.have_prec ? &Pb : nullptr, cols, b.Bbot, 1.0 / c.delta, pnorm, sigma_l, true, s);
    unpack_cols(b.Xp, b.kp, c.n, kg, Z + (size_t)g0 * ldz, ldz, s);
    for (auto& cs : cols) {
      if (cs.eta > c.o.tol_ne) status = APLICUR_W_MAXITER;
      eta_max = std::max(eta_max, cs.eta);
      iters = std::max(iters, cs.used);
      phases = std::max(phases, cs.phases);
    }
  }
  if (blocked) blk_apply(c, 0, Z, ldz, nrhs, dB, lddb, s);  // dB = A Z
  for (int k = 0; !blocked && k < nrhs; ++k) {
    const double* g = G + (size_t)k * ldg;
    double* z = Z + (size_t)k * ldz;
    fill(z, c.n, 0.0, s);
    ColState cs;
    cs.atb = vec_norm_n(c, g, s);
    if (!std::isfinite(cs.atb)) throw Error(APLICUR_E_BREAKDOWN, "non-finite values in G");
    if (cs.atb > 0.0)
      refine(c, P, Rhs{nullptr, g, 1.0 / c.delta}, z, cs, pnorm, sigma_l, true, nullptr, nullptr, s);
    else
      cs.eta = 0.0;
    if (cs.eta > c.o.tol_ne) status = APLICUR_W_MAXITER;
    eta_max = std::max(eta_max, cs.eta);
    iters = std::max(iters, cs.used);
    phases = std::max(phases, cs.phases);
    // dB = A z
    double* db = dB + (size_t)k * lddb;
    fill(db, c.m, 0.0, s);
    op_matvec(c.op, 0, z, db, c.st_mv, c.wk, s);
  }
  if (dA) {
    // R = B - A X (m x k), then the rank-2k gradient
    if (blocked) ensure_blk(c, blk_kp(std::min(nrhs, kBlkMaxCols)), s);  // no allocation while work lives
    bool owned = false;
    // dense A: [R, -AZ] (m x 2k) and [Z, X] (n x 2k) for one rank-2k product
    const size_t extra = c.op.csr ? 0 : (size_t)c.n * nrhs * 2;
    double* work = (double*)c.arena.transient(sizeof(double) * ((size_t)c.m * nrhs * 2 + extra), owned);
    try {
      double* R = work;                         // m x k, then -AZ in the next k columns
      double* AX = work + (size_t)c.m * nrhs;
      if (blocked) {
        blk_apply(c, 0, X, ldx, nrhs, AX, c.m, s);
      } else {
        for (int k = 0; k < nrhs; ++k) {
          fill(AX + (size_t)k * c.m, c.m, 0.0, s);
          op_matvec(c.op, 0, X + (size_t)k * ldx, AX + (size_t)k * c.m, c.st_mv, c.wk, s);
        }
      }
      sub_cols(B, ldb, AX, c.m, R, c.m, c.m, nrhs, s);
      if (c.op.csr) {
        grad_csr(c.op.row_ptr, c.op.col_idx, c.m, nrhs, R, c.m, Z, ldz, dB, lddb, X, ldx, dA, s);
      } else {
        copy_block(dB, lddb, AX, c.m, (int)c.m, nrhs, -1.0, s);  // AX <- -AZ
        double* ZX = work + (size_t)c.m * nrhs * 2;
        copy_block(Z, ldz, ZX, c.n, (int)c.n, nrhs, 1.0, s);
        copy_block(X, ldx, ZX + (size_t)c.n * nrhs, c.n, (int)c.n, nrhs, 1.0, s);
        if (c.A.format == APLICUR_DENSE_COL)
          // column-major dA (m x n) = R Z^T - (AZ) X^T = [R, -AZ] [Z, X]^T
          gemm(c, Op::N, Op::T, c.m, c.n, 2 * nrhs, 1.0, R, c.m, ZX, c.n, 0.0, dA, ldda);
        else
          // row-major dA is the column-major n x m matrix dA^T = [Z, X] [R, -AZ]^T
          gemm(c, Op::N, Op::T, c.n, c.m, 2 * nrhs, 1.0, ZX, c.n, R, c.m, 0.0, dA, ldda);
      }
      APL_HIP(hipGetLastError());
      APL_HIP(hipStreamSynchronize(s));
    } catch (...) {
      if (owned) {
        SyncGuard g(g_capture_mu);
        (void)hipFree(work);
      }
      throw;
    }
    if (owned) {
      SyncGuard g(g_capture_mu);
      APL_HIP(hipFree(work));
    }
  }
  APL_HIP(hipGetLastError());
  APL_HIP(hipStreamSynchronize(s));
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->status = status;
    info->phases = phases;
    info->iters = iters;
    info->rank = c.rank;
    info->eta = eta_max;
    info->sigma_hat = c.p_target;
    info->t_lsqr_ms = ms_since(t0);
    if (blocked) info->phases_bf16 = c.blk->phases16;
  }
  return status;
}

// Workspace of a context for solves (and adjoint solves) with up to nrhs
// columns: its set-up buffers, the blocked path's buffers for that many
// columns, and the adjoint's transient residual block.
static size_t workspace_for(const aplicur_mat* A, const aplicur_opts* o, int nrhs, hipStream_t s) {
  std::unique_ptr<Ctx> c(create(A, o, s));
  if (use_blocked(*c, nrhs)) ensure_blk(*c, blk_kp(std::min(nrhs, kBlkMaxCols)), s);
  APL_HIP(hipStreamSynchronize(s));
  // the adjoint's transient block: [R, -AZ] (m x 2k) and, for a dense A, [Z, X] (n x 2k)
  const size_t adj = Arena::aligned(sizeof(double) * ((size_t)c->m * nrhs * 2 + (c->op.csr ? 0 : (size_t)c->n * nrhs * 2)));
  return std::max(c->arena.peak, c->arena.used + adj);
}

// ------------------------------------------------------------------ batched solves
// Independent problems, largest first (by stored entries), taken from a
// shared counter by `workers` host threads; each thread owns a HIP stream
// (default priority) that first waits for the caller's stream, and runs
// whole problems on it (context, solve, release).  Every problem uses the
// same kernels as aplicur_solve; with the graphs option its LSQR iterations
// replay as captured graphs on that stream.  Returns after all streams are
// done; the first error (in problem order) is rethrown.
static int batched_workers(int batch, const aplicur_opts& o) {
  return std::max(1, std::min(batch, o.workers > 0 ? o.workers : 4));
}

// Bytes of one worker's slice of a batched call's workspace: the largest
// context any of the problems needs (each measured as aplicur_workspace_bytes
// does), rounded to the arena alignment.
static size_t batched_slice_bytes(int batch, const aplicur_mat* A, int nrhs, const aplicur_opts& o, hipStream_t s) {
  size_t slice = 0;
  for (int p = 0; p < batch; ++p) slice = std::max(slice, workspace_for(&A[p], &o, nrhs, s));
  return Arena::aligned(slice);
}

static int solve_batched(int batch, const aplicur_mat* A, const double* const* B, const int64_t* ldb, int nrhs,
                         double* const* X, const int64_t* ldx, const aplicur_opts& o, aplicur_info* info,
                         void* ws, size_t ws_bytes, hipStream_t caller) {
  for (int p = 0; p < batch; ++p) validate(&A[p], &o);
  const int workers = batched_workers(batch, o);
  // with a caller workspace, worker w carves every context it runs from
  // slice w; the slice fits the largest problem's context
  size_t slice = 0;
  if (ws) {
    slice = batched_slice_bytes(batch, A, nrhs, o, caller);
    APL_REQUIRE(ws_bytes >= slice * (size_t)workers,
                "the workspace needs " + std::to_string(slice * (size_t)workers) + " bytes (" +
                    std::to_string(workers) + " workers x " + std::to_string(slice) + ")");
  }
  std::vector<int> order(batch);
  std::iota(order.begin(), order.end(), 0);
  auto work = [&](int p) {
    return A[p].format == APLICUR_CSR ? (double)A[p].nnz : (double)A[p].m * (double)A[p].n;
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(a) > work(b); });
  int dev = 0;
  APL_HIP(hipGetDevice(&dev));
  hipEvent_t ready = nullptr;
  APL_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
  APL_HIP(hipEventRecord(ready, caller));
  std::atomic<int> next{0};
  std::vector<int> status(batch, APLICUR_OK), code(batch, 0);
  std::vector<std::string> msg(batch);
  auto worker = [&](int wid) {
    hipStream_t s = nullptr;
    char* my_ws = ws ? (char*)ws + slice * (size_t)wid : nullptr;
    bool ok;
    {
      SyncGuard g(g_capture_mu);
      ok = hipSetDevice(dev) == hipSuccess && hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess &&
           hipStreamWaitEvent(s, ready, 0) == hipSuccess;
    }
    if (!ok) {
      const int i = next.fetch_add(1);
      if (i < batch) {
        code[order[i]] = APLICUR_E_HIP;
        msg[order[i]] = "could not set up a worker stream";
      }
      if (s) (void)hipStreamDestroy(s);
      return;
    }
    for (;;) {
      const int i = next.fetch_add(1);
      if (i >= batch) break;
      const int p = order[i];
      Ctx* c = nullptr;
      try {
        c = create(&A[p], &o, s, my_ws, my_ws ? slice : 0);
        status[p] = solve(*c, B[p], ldb[p], nrhs, X[p], ldx[p], false, info ? &info[p] : nullptr, s);
      } catch (const Error& e) {
        code[p] = e.code;
        msg[p] = e.what();
      } catch (const std::exception& e) {
        code[p] = APLICUR_E_HIP;
        msg[p] = e.what();
      }
      delete c;
    }
    (void)hipStreamSynchronize(s);
    SyncGuard g(g_capture_mu);
    (void)hipStreamDestroy(s);
  };
  std::vector<std::thread> pool;
  for (int w = 1; w < workers; ++w) pool.emplace_back(worker, w);
  worker(0);
  for (auto& t : pool) t.join();
  (void)hipEventDestroy(ready);
  int worst = APLICUR_OK;
  for (int p = 0; p < batch; ++p) {
    if (code[p] != 0) throw Error(code[p], "problem " + std::to_string(p) + ": " + msg[p]);
    worst = std::max(worst, status[p]);
  }
  return worst;
}

}  // namespace aplicur

// ==================================================================== C ABI
using namespace aplicur;

struct aplicur_ctx {
  Ctx* impl;
};

template <class F>
static int guarded(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return APLICUR_E_HIP;
  } catch (...) {
    g_last_error = "unknown error";
    return APLICUR_E_HIP;
  }
}

extern "C" {

void aplicur_opts_default(aplicur_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->block = 20;
  o->r_probes = 10;
  o->seed = 7;
  o->mu = 0.0;
  o->eps_cur = -1.0;
  o->nu_prec = 10.0;
  o->nu_lsqr = 100.0;
  o->eps_lsqr = 1e-10;
  o->tol_ne = 1e-8;
  o->max_iter = 100000;
  o->max_rank = 0;
  o->precond = 1;
  o->precision = 0;
  o->max_outer = 0;
  o->xi = 8;
}

int aplicur_sketch(const aplicur_mat* A, const aplicur_opts* opts, void* ws, size_t ws_bytes, void* stream,
                   aplicur_ctx** ctx_out) {
  return guarded([&]() {
    APL_REQUIRE(ctx_out, "ctx_out is null");
    *ctx_out = nullptr;
    APL_REQUIRE(!ws || ws_bytes > 0, "ws_bytes must be > 0 with a workspace");
    APL_REQUIRE(((uintptr_t)ws % Arena::kAlign) == 0, "the workspace must be 256-byte aligned");
    Ctx* c = create(A, opts, (hipStream_t)stream, ws, ws ? ws_bytes : 0);
    *ctx_out = new aplicur_ctx{c};
    return APLICUR_OK;
  });
}

int64_t aplicur_workspace_bytes(const aplicur_mat* A, int32_t nrhs, const aplicur_opts* opts, void* stream) {
  int64_t bytes = 0;
  const int rc = guarded([&]() {
    APL_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
    bytes = (int64_t)workspace_for(A, opts, nrhs, (hipStream_t)stream);
    return APLICUR_OK;
  });
  return rc == APLICUR_OK ? bytes : (int64_t)rc;
}

int aplicur_solve(aplicur_ctx* ctx, const double* B, int64_t ldb, int32_t nrhs, double* X, int64_t ldx,
                  int32_t x_is_warm, aplicur_info* info, void* stream) {
  return guarded([&]() {
    APL_REQUIRE(ctx && ctx->impl, "null context");
    return solve(*ctx->impl, B, ldb, nrhs, X, ldx, x_is_warm != 0, info, (hipStream_t)stream);
  });
}

int64_t aplicur_batched_workspace_bytes(int32_t batch, const aplicur_mat* A, int32_t nrhs, const aplicur_opts* opts,
                                        void* stream) {
  int64_t bytes = 0;
  const int rc = guarded([&]() {
    APL_REQUIRE(batch >= 1 && A && opts, "need batch >= 1 problems and options");
    APL_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
    for (int p = 0; p < batch; ++p) validate(&A[p], opts);
    const size_t slice = batched_slice_bytes(batch, A, nrhs, *opts, (hipStream_t)stream);
    bytes = (int64_t)(slice * (size_t)batched_workers(batch, *opts));
    return APLICUR_OK;
  });
  return rc == APLICUR_OK ? bytes : (int64_t)rc;
}

int aplicur_solve_batched(int32_t batch, const aplicur_mat* A, const double* const* B, const int64_t* ldb,
                          int32_t nrhs, double* const* X, const int64_t* ldx, const aplicur_opts* opts,
                          void* ws, size_t ws_bytes, aplicur_info* info, void* stream) {
  return guarded([&]() {
    APL_REQUIRE(batch >= 0, "batch must be >= 0");
    if (batch == 0) return (int)APLICUR_OK;
    APL_REQUIRE(A && B && ldb && X && ldx && opts, "null batch arrays");
    APL_REQUIRE(!ws || ws_bytes > 0, "ws_bytes must be > 0 with a workspace");
    APL_REQUIRE(((uintptr_t)ws % Arena::kAlign) == 0, "the workspace must be 256-byte aligned");
    return solve_batched(batch, A, B, ldb, nrhs, X, ldx, *opts, info, ws, ws ? ws_bytes : 0, (hipStream_t)stream);
  });
}

int aplicur_solve_backward(aplicur_ctx* ctx, const double* X, int64_t ldx, const double* B, int64_t ldb,
                           const double* G, int64_t ldg, int32_t nrhs, double* Z, int64_t ldz, double* dB,
                           int64_t lddb, double* dA, int64_t ldda, aplicur_info* info, void* stream) {
  return guarded([&]() -> int {
    APL_REQUIRE(ctx && ctx->impl, "null context");
    return solve_backward(*ctx->impl, X, ldx, B, ldb, G, ldg, nrhs, Z, ldz, dB, lddb, dA, ldda, info,
                          (hipStream_t)stream);
  });
}

int aplicur_matvec(aplicur_ctx* ctx, int32_t trans, const double* x, double* y, void* stream) {
  return guarded([&]() {
    APL_REQUIRE(ctx && ctx->impl && x && y, "null argument");
    Ctx& c = *ctx->impl;
    hipStream_t s = (hipStream_t)stream;
    if (!trans) fill(y, c.m, 0.0, s);
    op_matvec(c.op, trans, x, y, c.st_mv, c.wk, s);
    APL_HIP(hipGetLastError());
    return APLICUR_OK;
  });
}

int aplicur_matmat(aplicur_ctx* ctx, int32_t trans, const double* X, int64_t ldx, int32_t k, double* Y, int64_t ldy,
                   int32_t prec, void* stream) {
  return guarded([&]() {
    APL_REQUIRE(ctx && ctx->impl && X && Y, "null argument");
    Ctx& c = *ctx->impl;
    APL_REQUIRE(k >= 1, "k must be >= 1");
    APL_REQUIRE(prec >= 0 && prec <= 2, "prec must be 0, 1 or 2");
    APL_REQUIRE(prec == 0 || (!c.op.csr && c.fp32), "prec 1 needs a dense A and a context of precision 1 or 2");
    APL_REQUIRE(prec < 2 || c.bf16, "prec 2 needs a context of precision 2");
    APL_REQUIRE(ldx >= (trans ? c.m : c.n) && ldy >= (trans ? c.n : c.m), "leading dimensions too small");
    hipStream_t s = (hipStream_t)stream;
    set_stream(c, s);
    if (c.op.csr) {
      for (int j = 0; j < k; ++j) {
        double* y = Y + (size_t)j * ldy;
        if (!trans) fill(y, c.m, 0.0, s);
        op_matvec(c.op, trans, X + (size_t)j * ldx, y, c.st_mv, c.wk, s);
      }
    } else {
      blk_apply(c, trans, X, ldx, k, Y, ldy, s, prec);
    }
    APL_HIP(hipGetLastError());
    return APLICUR_OK;
  });
}

int aplicur_precond_apply(aplicur_ctx* ctx, int32_t trans, const double* z, double* y, void* stream) {
  return guarded([&]() {
    APL_REQUIRE(ctx && ctx->impl && z && y, "null argument");
    Ctx& c = *ctx->impl;
    APL_REQUIRE(c.have_prec, "no preconditioner has been built (run aplicur_solve with precond 1 or 2 first)");
    set_stream(c, (hipStream_t)stream);
    ensure_vhat(c, (hipStream_t)stream);
    gk_precond_apply(c.op, c.prec, trans != 0, z, y, (hipStream_t)stream);
    APL_HIP(hipGetLastError());
    return APLICUR_OK;
  });
}

int aplicur_time_product(aplicur_ctx* ctx, int32_t trans, const double* x, double* y, int32_t reps, void* flush,
                         int64_t flush_bytes, void* stream, double* us_per_launch) {
  return guarded([&]() {
    APL_REQUIRE(ctx && ctx->impl && x && y && us_per_launch && reps >= 1, "bad argument");
    APL_REQUIRE(!flush || (flush_bytes >= 16 && flush_bytes % 16 == 0), "flush_bytes must be a positive multiple of 16");
    Ctx& c = *ctx->impl;
    hipStream_t s = (hipStream_t)stream;
    // y (m) = A x - y ; scratch (n) = A^T y, alternating as in the LSQR loop
    fill(y, c.m, 0.0, s);
    op_matvec(c.op, 0, x, y, c.st_mv, c.wk, s);
    op_matvec(c.op, 1, y, c.g, c.st_mv, c.wk, s);
    std::vector<hipEvent_t> ev(2 * (size_t)reps);
    for (auto& e : ev) APL_HIP(hipEventCreate(&e));
    for (int i = 0; i < reps; ++i) {
      if (flush) touch_buffer(flush, flush_bytes, s);
      if (!trans) {
        op_matvec(c.op, 0, x, y, c.st_mv, c.wk, s, ev[2 * i], ev[2 * i + 1]);
        op_matvec(c.op, 1, y, c.g, c.st_mv, c.wk, s);
      } else {
        op_matvec(c.op, 0, x, y, c.st_mv, c.wk, s);
        op_matvec(c.op, 1, y, c.g, c.st_mv, c.wk, s, ev[2 * i], ev[2 * i + 1]);
      }
    }
    APL_HIP(hipEventSynchronize(ev.back()));
    double tot = 0.0;
    for (int i = 0; i < reps; ++i) {
      float ms = 0.f;
      APL_HIP(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]));
      tot += ms;
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    APL_HIP(hipGetLastError());
    *us_per_launch = 1e3 * tot / reps;
    return APLICUR_OK;
  });
}

int aplicur_time_matmat(aplicur_ctx* ctx, int32_t trans, const double* X, int64_t ldx, int32_t k, double* Y,
                        int64_t ldy, int32_t prec, int32_t reps, void* flush, int64_t flush_bytes, void* stream,
                        double* us_per_launch) {
  return guarded([&]() {
    APL_REQUIRE(ctx && ctx->impl && X && Y && us_per_launch && reps >= 1, "bad argument");
    Ctx& c = *ctx->impl;
    APL_REQUIRE(!c.op.csr, "aplicur_time_matmat needs a dense A");
    APL_REQUIRE(k >= 1 && k <= kBlkMaxCols, "k must be in [1, 64]");
    APL_REQUIRE(prec >= 0 && prec <= 2, "prec must be 0, 1 or 2");
    APL_REQUIRE(prec == 0 || c.fp32, "prec 1 needs a context of precision 1 or 2");
    APL_REQUIRE(prec < 2 || c.bf16, "prec 2 needs a context of precision 2");
    APL_REQUIRE(ldx >= (trans ? c.m : c.n) && ldy >= (trans ? c.n : c.m), "leading dimensions too small");
    APL_REQUIRE(!flush || (flush_bytes >= 16 && flush_bytes % 16 == 0), "flush_bytes must be a positive multiple of 16");
    hipStream_t s = (hipStream_t)stream;
    set_stream(c, s);
    blk_apply(c, trans, X, ldx, k, Y, ldy, s, prec);  // copies made on first use, before the timed launches
    std::vector<hipEvent_t> ev(2 * (size_t)reps);
    for (auto& e : ev) APL_HIP(hipEventCreate(&e));
    for (int i = 0; i < reps; ++i) {
      if (flush) touch_buffer(flush, flush_bytes, s);
      blk_apply(c, trans, X, ldx, k, Y, ldy, s, prec, ev[2 * i], ev[2 * i + 1]);
    }
    APL_HIP(hipEventSynchronize(ev.back()));
    double tot = 0.0;
    for (int i = 0; i < reps; ++i) {
      float ms = 0.f;
      APL_HIP(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]));
      tot += ms;
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    APL_HIP(hipGetLastError());
    *us_per_launch = 1e3 * tot / reps;
    return APLICUR_OK;
  });
}

int64_t aplicur_ctx_query(const aplicur_ctx* ctx, int32_t what, void* host_out, size_t bytes) {
  if (!ctx || !ctx->impl) {
    g_last_error = "null context";
    return APLICUR_E_INVALID;
  }
  Ctx& c = *ctx->impl;
  try {
    std::vector<char> buf;
    auto put = [&](const void* p, size_t nb) { buf.assign((const char*)p, (const char*)p + nb); };
    auto dev = [&](const void* p, size_t nb) {
      buf.resize(nb);
      if (nb) {
        APL_HIP(hipDeviceSynchronize());
        APL_HIP(hipMemcpy(buf.data(), p, nb, hipMemcpyDeviceToHost));
      }
    };
    switch (what) {
      case 1: dev(c.Y, sizeof(double) * (size_t)c.s * c.n); break;
      case 2: case 3: {
        if (c.o.sketch >= 1) {  // Gaussian sketch: no sparse sign structure
          buf.clear();
          break;
        }
        std::vector<uint16_t> rows((size_t)c.m * c.xi);
        std::vector<uint8_t> neg(c.m);
        APL_HIP(hipDeviceSynchronize());
        if (c.S_rows) {
          APL_HIP(hipMemcpy(rows.data(), c.S_rows, rows.size() * 2, hipMemcpyDeviceToHost));
          APL_HIP(hipMemcpy(neg.data(), c.S_neg, neg.size(), hipMemcpyDeviceToHost));
        }
        std::vector<int32_t> out((size_t)c.m * c.xi);
        for (long long i = 0; i < c.m; ++i)
          for (int t = 0; t < c.xi; ++t)
            out[(size_t)i * c.xi + t] = (what == 2) ? rows[(size_t)i * c.xi + t] : (((neg[i] >> t) & 1) ? -1 : 1);
        put(out.data(), out.size() * 4);
        break;
      }
      case 4: dev(c.W, sizeof(double) * (size_t)c.n * c.r); break;
      case 5: put(c.J.data(), c.J.size() * 4); break;
      case 6: put(c.I.data(), c.I.size() * 4); break;
      case 7: put(c.rho_hist.data(), c.rho_hist.size() * 8); break;
      case 8: put(c.rank_hist.data(), c.rank_hist.size() * 4); break;
      case 9: put(c.rebuild_hist.data(), c.rebuild_hist.size() * 4); break;
      case 10: {
        int64_t sz[7] = {c.m, c.n, c.s, c.xi, c.rank, (int64_t)c.rank_hist.size(), c.r};
        put(sz, sizeof(sz));
        break;
      }
      case 11: put(c.p_sigma_host.data(), c.p_sigma_host.size() * 8); break;
      case 12: put(c.phase_iters0.data(), c.phase_iters0.size() * 4); break;
      case 13: put(c.phase_eta0.data(), c.phase_eta0.size() * 8); break;
      case 14: put(c.sweep_hist.data(), c.sweep_hist.size() * 4); break;
      case 15:
        if (c.o.precond == 2 && c.have_prec) dev(c.M2, sizeof(double) * (size_t)c.prec.ell * c.prec.ell);
        else buf.clear();
        break;
      default: g_last_error = "unknown query"; return APLICUR_E_INVALID;
    }
    if (host_out && bytes) std::memcpy(host_out, buf.data(), std::min(bytes, buf.size()));
    return (int64_t)buf.size();
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.code;
  }
}

void aplicur_ctx_destroy(aplicur_ctx* ctx) {
  if (!ctx) return;
  delete ctx->impl;
  delete ctx;
}

const char* aplicur_last_error(void) { return g_last_error.c_str(); }
const char* aplicur_version(void) { return "aplicur-gfx950 0.1"; }

}  // extern "C"
