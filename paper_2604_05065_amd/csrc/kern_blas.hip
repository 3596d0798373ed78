// Dense FP64 BLAS-3 of the set-up, hand-written for gfx950 (see blas.h):
// GEMM on the FP64 16x16x4 MFMA with LDS-staged 128 x 128 output tiles,
// blocked triangular solves, a fixed-order 2-norm, and the Gaussian sketch
// product with FP32 or BF16 inputs and FP64 accumulation.
#include <algorithm>
#include <cmath>
#include <vector>

#include "blas.h"

namespace aplicur {

typedef double f64x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

// ============================================================== GEMM
// Workgroup (bx, by, bz) owns the output tile rows [128 bx, +128), columns
// [128 by, +128) and the k chunk bz.  Each 16-deep stage of op(A) (128 x 16)
// and op(B) (16 x 128) is loaded into registers (8 values per thread, the
// next stage's loads in flight during the current stage's MFMAs), stored to
// LDS as [k][row] / [k][column], and wave (wr, wc) = (w / 2, w % 2) takes the
// 64 x 64 quarter [64 wr, +64) x [64 wc, +64) as 4 x 4 MFMA tiles.  MFMA
// operands: A lane (i, q) = op(A)(i, q), B lane (i, q) = op(B)(q, i); D lane
// (i, q) register r = row q + 4 r, column i.
constexpr int kGM = 128;      // tile rows and columns
constexpr int kGKs = 16;      // k per stage
constexpr int kGThreads = 256;
constexpr int kGPad = 2;      // LDS row padding (doubles)

// Registers of one stage of a 128 x 16 operand tile.  Element (i, kk) of the
// operand (i < 128 the tile row, kk < 16 the stage's k) lives at X[i + kk ld]
// (KC = false: rows contiguous) or X[kk + i ld] (KC = true: k contiguous).
// tile_load only issues the loads (addresses clamped into range) so that
// they stay in flight during the MFMAs of the current stage; tile_store
// zeroes the out-of-range entries when it writes the stage to LDS.
typedef double f64x2_t __attribute__((ext_vector_type(2)));

template <bool KC, class T>
__device__ __forceinline__ void tile_load(const T* __restrict__ X, long long ld, long long rows, long long i0,
                                          long long k0, long long kend, T (&r)[8], bool vec) {
  const int t = threadIdx.x;
  if constexpr (sizeof(T) == 8) {
    // whole stage in range and 16-byte aligned rows: four 16-byte loads
    if (vec && i0 + kGM <= rows && k0 + kGKs <= kend) {
      const T* p = KC ? X + (i0 + t / 2) * ld + k0 + (t % 2) * 8 : X + (k0 + t / 16) * ld + i0 + (t % 16) * 8;
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const f64x2_t u = ((const f64x2_t*)p)[h];
        r[2 * h] = u.x;
        r[2 * h + 1] = u.y;
      }
      return;
    }
  }
  if (!KC) {
    const long long kk = k0 + t / 16;
    const long long ib = i0 + (t % 16) * 8;
    const T* p = X + (kk < kend ? kk : 0) * ld;
#pragma unroll
    for (int e = 0; e < 8; ++e) r[e] = p[ib + e < rows ? ib + e : 0];
  } else {
    const long long i = i0 + t / 2;
    const long long kb = k0 + (t % 2) * 8;
    const T* p = X + (i < rows ? i : 0) * ld;
#pragma unroll
    for (int e = 0; e < 8; ++e) r[e] = p[kb + e < kend ? kb + e : 0];
  }
}

template <bool KC, class T, int LD>
__device__ __forceinline__ void tile_store(T (*Xs)[LD], const T (&r)[8], long long rows, long long i0, long long k0,
                                           long long kend) {
  const int t = threadIdx.x;
  if (!KC) {
    const int kk = t / 16, ib = (t % 16) * 8;
    const bool kin = k0 + kk < kend;
#pragma unroll
    for (int e = 0; e < 8; ++e) Xs[kk][ib + e] = (kin && i0 + ib + e < rows) ? r[e] : (T)0;
  } else {
    const int i = t / 2, kb = (t % 2) * 8;
    const bool iin = i0 + i < rows;
#pragma unroll
    for (int e = 0; e < 8; ++e) Xs[kb + e][i] = (iin && k0 + kb + e < kend) ? r[e] : (T)0;
  }
}

// Two waves per SIMD (at most 256 registers, 128 of them the accumulators),
// so that one wave's MFMAs overlap the other's LDS reads and barriers.
template <bool TA, bool TB>
__global__ void __launch_bounds__(kGThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
    k_dgemm(long long M, long long N, long long K, long long kchunk, double alpha, const double* __restrict__ A,
            long long lda, const double* __restrict__ B, long long ldb, double beta, double* __restrict__ C,
            long long ldc, double* __restrict__ part, int vec_a, int vec_b) {
  __shared__ double As[kGKs][kGM + kGPad];
  __shared__ double Bs[kGKs][kGM + kGPad];
  const long long i0 = (long long)blockIdx.x * kGM, j0 = (long long)blockIdx.y * kGM;
  const long long kbeg = (long long)blockIdx.z * kchunk;
  const long long kend = min(K, kbeg + kchunk);
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int li = lane % 16, lq = lane / 16;
  const int wr = wave / 2, wc = wave % 2;
  f64x4_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f64x4_t{0.0, 0.0, 0.0, 0.0};
  double ra[8], rb[8];
  if (kbeg < kend) {
    tile_load<TA>(A, lda, M, i0, kbeg, kend, ra, vec_a != 0);
    tile_load<!TB>(B, ldb, N, j0, kbeg, kend, rb, vec_b != 0);
  }
  for (long long k0 = kbeg; k0 < kend; k0 += kGKs) {
    __syncthreads();
    tile_store<TA, double, kGM + kGPad>(As, ra, M, i0, k0, kend);
    tile_store<!TB, double, kGM + kGPad>(Bs, rb, N, j0, k0, kend);
    __syncthreads();
    if (k0 + kGKs < kend) {
      tile_load<TA>(A, lda, M, i0, k0 + kGKs, kend, ra, vec_a != 0);
      tile_load<!TB>(B, ldb, N, j0, k0 + kGKs, kend, rb, vec_b != 0);
    }
#pragma unroll
    for (int kk = 0; kk < kGKs; kk += 4) {
      double a[4], b[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        a[t] = As[kk + lq][wr * 64 + t * 16 + li];
        b[t] = Bs[kk + lq][wc * 64 + t * 16 + li];
      }
#pragma unroll
      for (int ti = 0; ti < 4; ++ti)
#pragma unroll
        for (int tj = 0; tj < 4; ++tj)
          acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ti], b[tj], acc[ti][tj], 0, 0, 0);
    }
  }
  double* out = part ? part + (long long)blockIdx.z * M * N : nullptr;
#pragma unroll
  for (int ti = 0; ti < 4; ++ti)
#pragma unroll
    for (int tj = 0; tj < 4; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long long row = i0 + wr * 64 + ti * 16 + lq + 4 * r;
        const long long col = j0 + wc * 64 + tj * 16 + li;
        if (row < M && col < N) {
          const double v = acc[ti][tj][r];
          if (out) {
            out[row + col * M] = v;
          } else {
            double* c = C + row + col * ldc;
            *c = beta == 0.0 ? alpha * v : alpha * v + beta * *c;
          }
        }
      }
}

// C = alpha * (sum of the parts in order) + beta * C
__global__ void __launch_bounds__(kBlock)
    k_gemm_reduce(const double* __restrict__ part, int parts, long long M, long long N, double alpha, double beta,
                  double* C, long long ldc) {
  const long long mn = M * N;
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < mn; e += (long long)gridDim.x * kBlock) {
    double acc = 0.0;
    for (int p = 0; p < parts; ++p) acc += part[(long long)p * mn + e];
    double* c = C + e % M + (e / M) * ldc;
    *c = beta == 0.0 ? alpha * acc : alpha * acc + beta * *c;
  }
}

// k chunks for a shape.  Two workgroups of k_dgemm fit a CU (waves_per_eu 2),
// so kGConcurrent of them run at once and a launch takes about
// ceil(tiles parts / kGConcurrent) rounds of kchunk-deep tiles; each part
// beyond the first adds a plane of the output written and read again.  The
// count (1 to 64, chunks of at least 256, a multiple of the stage depth)
// minimises that estimate: MFMA time per round and k from the FP64 peak at
// about 0.7 (kGRoundUsPerK), plane traffic at about 5 TB/s.  A function of the
// shape only.
constexpr long long kGConcurrent = 512;
constexpr double kGRoundUsPerK = 0.3;
constexpr double kGPlaneUsPerWord = 8.0 / 5.0e6;
static int gemm_chunks(long long m, long long n, long long k, long long* kchunk) {
  const long long tiles = ((m + kGM - 1) / kGM) * ((n + kGM - 1) / kGM);
  const long long pmax = std::max<long long>(1, std::min<long long>(64, k / 256));
  long long best_p = 1, best_kc = (k + kGKs - 1) / kGKs * kGKs;
  double best = INFINITY;
  for (long long p = 1; p <= pmax; ++p) {
    const long long kc = ((k + p - 1) / p + kGKs - 1) / kGKs * kGKs;
    const long long parts = (k + kc - 1) / kc;
    const long long rounds = (tiles * parts + kGConcurrent - 1) / kGConcurrent;
    double cost = (double)rounds * (double)kc * kGRoundUsPerK;
    if (parts > 1) cost += (double)(2 * parts + 1) * (double)(m * n) * kGPlaneUsPerWord;
    if (cost < best * 0.98) {  // more parts only for a clear gain
      best = cost;
      best_p = parts;
      best_kc = kc;
    }
  }
  *kchunk = best_kc;
  return (int)best_p;
}

size_t dgemm_work(Op ta, Op tb, long long m, long long n, long long k) {
  (void)ta;
  (void)tb;
  long long kc = 0;
  const int parts = gemm_chunks(m, n, k, &kc);
  return parts > 1 ? (size_t)parts * (size_t)(m * n) : 0;
}

void dgemm(Op ta, Op tb, long long m, long long n, long long k, double alpha, const double* A, long long lda,
           const double* B, long long ldb, double beta, double* C, long long ldc, double* work, size_t work_count,
           hipStream_t s) {
  if (m <= 0 || n <= 0) return;
  if (k <= 0) {
    // C = beta C
    hipLaunchKernelGGL(k_gemm_reduce, dim3(std::min<unsigned>(ceil_div(m * n, kBlock), 4096)), dim3(kBlock), 0, s,
                       (const double*)nullptr, 0, m, n, 0.0, beta, C, ldc);
    return;
  }
  long long kc = 0;
  int parts = gemm_chunks(m, n, k, &kc);
  if (parts > 1 && (!work || (size_t)parts * (size_t)(m * n) > work_count)) {
    // as many chunks as the scratch holds (a function of the shape and the
    // scratch size only)
    const long long fit = work ? (long long)(work_count / (size_t)(m * n)) : 1;
    parts = (int)std::max<long long>(1, std::min<long long>(parts, fit));
    kc = ((k + parts - 1) / parts + kGKs - 1) / kGKs * kGKs;
    parts = (int)((k + kc - 1) / kc);
  }
  const dim3 g((unsigned)((m + kGM - 1) / kGM), (unsigned)((n + kGM - 1) / kGM), (unsigned)parts);
  double* part = parts > 1 ? work : nullptr;
  const bool tA = ta == Op::T, tB = tb == Op::T;
  // 16-byte loads need even leading dimensions and 16-byte aligned bases
  // (the k chunks and tile origins are even)
  const int va = (lda % 2 == 0) && ((uintptr_t)A % 16 == 0);
  const int vb = (ldb % 2 == 0) && ((uintptr_t)B % 16 == 0);
  if (!tA && !tB)
    hipLaunchKernelGGL((k_dgemm<false, false>), g, dim3(kGThreads), 0, s, m, n, k, kc, alpha, A, lda, B, ldb, beta, C,
                       ldc, part, va, vb);
  else if (!tA && tB)
    hipLaunchKernelGGL((k_dgemm<false, true>), g, dim3(kGThreads), 0, s, m, n, k, kc, alpha, A, lda, B, ldb, beta, C,
                       ldc, part, va, vb);
  else if (tA && !tB)
    hipLaunchKernelGGL((k_dgemm<true, false>), g, dim3(kGThreads), 0, s, m, n, k, kc, alpha, A, lda, B, ldb, beta, C,
                       ldc, part, va, vb);
  else
    hipLaunchKernelGGL((k_dgemm<true, true>), g, dim3(kGThreads), 0, s, m, n, k, kc, alpha, A, lda, B, ldb, beta, C,
                       ldc, part, va, vb);
  if (parts > 1)
    hipLaunchKernelGGL(k_gemm_reduce, dim3(std::min<unsigned>(ceil_div(m * n, kBlock), 4096)), dim3(kBlock), 0, s,
                       (const double*)part, parts, m, n, alpha, beta, C, ldc);
}

// ============================================================== TRSM
// Diagonal blocks of op(T) of at most kTB x kTB in LDS; op(T)(i, j) is
// T[i + j ldt] (trans = 0) or T[j + i ldt] (trans = 1).  LOWER: op(T) is lower
// triangular (forward substitution for Left, backward over columns for Right).
constexpr int kTB = 64;

__device__ __forceinline__ void load_diag(double (*Ts)[kTB + 1], const double* T, long long ldt, int k, int trans) {
  for (int e = threadIdx.x; e < k * k; e += kBlock) {
    const int i = e % k, j = e / k;
    Ts[i][j] = trans ? T[j + (long long)i * ldt] : T[i + (long long)j * ldt];
  }
}

// Left: op(T) X = B for the k x ncols block B (k <= kTB): one wave per column,
// lane i holding x_i.  Column-oriented substitution: at step i the lane of
// the pivot finishes x_i (division by the diagonal), and every lane still to
// come subtracts op(T)(lane, i) x_i, so each x_j takes its terms in the order
// of i (ascending for LOWER, descending otherwise).
constexpr int kTrsmCols = kBlock / kWave;  // columns per workgroup
template <bool LOWER>
__global__ void __launch_bounds__(kBlock)
    k_trsm_left(int k, long long ncols, const double* __restrict__ T, long long ldt, int trans, int unit, double* B,
                long long ldb) {
  __shared__ double Ts[kTB][kTB + 1];
  load_diag(Ts, T, ldt, k, trans);
  __syncthreads();
  const int lane = threadIdx.x % kWave;
  const long long c = (long long)blockIdx.x * kTrsmCols + threadIdx.x / kWave;
  if (c >= ncols) return;  // whole waves leave together; no barrier follows
  double* col = B + c * ldb;
  double x = lane < k ? col[lane] : 0.0;
  if (LOWER) {
    for (int i = 0; i < k; ++i) {
      if (lane == i && !unit) x = x / Ts[i][i];
      const double xi = lane_bcast(x, i);
      if (lane > i && lane < k) x -= Ts[lane][i] * xi;
    }
  } else {
    for (int i = k - 1; i >= 0; --i) {
      if (lane == i && !unit) x = x / Ts[i][i];
      const double xi = lane_bcast(x, i);
      if (lane < i) x -= Ts[lane][i] * xi;
    }
  }
  if (lane < k) col[lane] = x;
}

// Right: X op(T) = B for the nrows x k block B (k <= kTB); thread = row.
// UPPER: x_j = (b_j - sum_{i<j} x_i op(T)(i,j)) / op(T)(j,j), j ascending;
// else j descending over i > j.
template <bool UPPER>
__global__ void __launch_bounds__(kBlock)
    k_trsm_right(int k, long long nrows, const double* __restrict__ T, long long ldt, int trans, int unit, double* B,
                 long long ldb) {
  __shared__ double Ts[kTB][kTB + 1];
  load_diag(Ts, T, ldt, k, trans);
  __syncthreads();
  const long long r = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (r >= nrows) return;
  double x[kTB];
#pragma unroll
  for (int j = 0; j < kTB; ++j) x[j] = j < k ? B[r + (long long)j * ldb] : 0.0;
  if (UPPER) {
#pragma unroll
    for (int j = 0; j < kTB; ++j) {
      if (j < k) {
        double acc = x[j];
#pragma unroll
        for (int i = 0; i < j; ++i) acc -= x[i] * Ts[i][j];
        x[j] = unit ? acc : acc / Ts[j][j];
      }
    }
  } else {
#pragma unroll
    for (int j = kTB - 1; j >= 0; --j) {
      if (j < k) {
        double acc = x[j];
#pragma unroll
        for (int i = j + 1; i < kTB; ++i)
          if (i < k) acc -= x[i] * Ts[i][j];
        x[j] = unit ? acc : acc / Ts[j][j];
      }
    }
  }
#pragma unroll
  for (int j = 0; j < kTB; ++j)
    if (j < k) B[r + (long long)j * ldb] = x[j];
}

__global__ void k_scale(double* B, long long ldb, long long rows, long long cols, double alpha) {
  const long long count = rows * cols;
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < count; e += (long long)gridDim.x * kBlock)
    B[e % rows + (e / rows) * ldb] *= alpha;
}

void dtrsm(Side side, Uplo uplo, Op trans, Diag diag, long long m, long long n, double alpha, const double* T,
           long long ldt, double* B, long long ldb, double* work, size_t work_count, hipStream_t s) {
  if (m <= 0 || n <= 0) return;
  if (alpha != 1.0)
    hipLaunchKernelGGL(k_scale, dim3(std::min<unsigned>(ceil_div(m * n, kBlock), 4096)), dim3(kBlock), 0, s, B, ldb,
                       m, n, alpha);
  const int tr = trans == Op::T ? 1 : 0, unit = diag == Diag::Unit ? 1 : 0;
  // op(T)'s sub-block (rows r0.., columns c0..) as a GEMM operand: T itself
  // at (r0, c0) when not transposed, else T^T of T's block at (c0, r0)
  auto sub = [&](long long r0, long long c0) { return tr ? T + c0 + r0 * ldt : T + r0 + c0 * ldt; };
  const Op opT = tr ? Op::T : Op::N;
  if (side == Side::Left) {
    const long long k = m;
    const bool lower = (uplo == Uplo::Lower) != (tr == 1);
    const long long nb = (k + kTB - 1) / kTB;
    for (long long q = 0; q < nb; ++q) {
      const long long blk = lower ? q : nb - 1 - q;
      const long long j0 = blk * kTB, jb = std::min<long long>(kTB, k - j0);
      const unsigned g = ceil_div(n, kTrsmCols);
      if (lower)
        hipLaunchKernelGGL(k_trsm_left<true>, dim3(g), dim3(kBlock), 0, s, (int)jb, n, sub(j0, j0), ldt, tr, unit,
                           B + j0, ldb);
      else
        hipLaunchKernelGGL(k_trsm_left<false>, dim3(g), dim3(kBlock), 0, s, (int)jb, n, sub(j0, j0), ldt, tr, unit,
                           B + j0, ldb);
      // the other rows: B_rest -= op(T)(rest, block) X_block
      if (lower && j0 + jb < k)
        dgemm(opT, Op::N, k - j0 - jb, n, jb, -1.0, sub(j0 + jb, j0), ldt, B + j0, ldb, 1.0, B + j0 + jb, ldb, work,
              work_count, s);
      if (!lower && j0 > 0)
        dgemm(opT, Op::N, j0, n, jb, -1.0, sub(0, j0), ldt, B + j0, ldb, 1.0, B, ldb, work, work_count, s);
    }
  } else {
    const long long k = n;
    const bool upper = (uplo == Uplo::Upper) != (tr == 1);
    const long long nb = (k + kTB - 1) / kTB;
    for (long long q = 0; q < nb; ++q) {
      const long long blk = upper ? q : nb - 1 - q;
      const long long j0 = blk * kTB, jb = std::min<long long>(kTB, k - j0);
      const unsigned g = ceil_div(m, kBlock);
      double* Bj = B + j0 * ldb;
      if (upper)
        hipLaunchKernelGGL(k_trsm_right<true>, dim3(g), dim3(kBlock), 0, s, (int)jb, m, sub(j0, j0), ldt, tr, unit, Bj,
                           ldb);
      else
        hipLaunchKernelGGL(k_trsm_right<false>, dim3(g), dim3(kBlock), 0, s, (int)jb, m, sub(j0, j0), ldt, tr, unit, Bj,
                           ldb);
      // the later columns: B(:, rest) -= X(:, block) op(T)(block, rest)
      if (upper && j0 + jb < k)
        dgemm(Op::N, opT, m, k - j0 - jb, jb, -1.0, Bj, ldb, sub(j0, j0 + jb), ldt, 1.0, B + (j0 + jb) * ldb, ldb,
              work, work_count, s);
      if (!upper && j0 > 0)
        dgemm(Op::N, opT, m, j0, jb, -1.0, Bj, ldb, sub(j0, 0), ldt, 1.0, B, ldb, work, work_count, s);
    }
  }
}

// ============================================================== 2-norm
__global__ void __launch_bounds__(kBlock) k_sumsq_parts(long long n, const double* __restrict__ x, double* parts) {
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
    acc += x[i] * x[i];
  acc = block_sum(acc);
  if (threadIdx.x == 0) parts[blockIdx.x] = acc;
}

__global__ void __launch_bounds__(kBlock) k_sum_parts(const double* parts, int count, double* out) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < count; i += kBlock) acc += parts[i];
  acc = block_sum(acc);
  if (threadIdx.x == 0) out[0] = acc;
}

double dnrm2(long long n, const double* x, double* tmp, hipStream_t s) {
  if (n <= 0) return 0.0;
  hipLaunchKernelGGL(k_sumsq_parts, dim3(kNrm2Parts), dim3(kBlock), 0, s, n, x, tmp);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(kBlock), 0, s, (const double*)tmp, kNrm2Parts, tmp + kNrm2Parts);
  double h = 0.0;
  APL_HIP(hipMemcpyAsync(&h, tmp + kNrm2Parts, sizeof(double), hipMemcpyDeviceToHost, s));
  APL_HIP(hipStreamSynchronize(s));
  return std::sqrt(h);
}

// ============================================================== Gaussian sketch product, FP32 / BF16 inputs
// Y^T (n x s, column-major = Y row-major) = A_cm (n x m) S^T: output tile
// rows [128 bx, +128) of the n columns of A, columns [128 by, +128) of the s
// sketch rows; the m-long reduction in 32-deep stages.  Operand element (i,
// kk): A at A[kk lda + i], S^T at S[j + kk s] (both rows contiguous).
// FP32: each stage runs 8 FP32 16x16x4 MFMAs per tile into a zeroed FP32
// accumulator (two 16-term sums), added to the FP64 accumulator after each
// 16 terms.  BF16: one 16x16x32 BF16 MFMA per tile and stage (32 terms
// exact products, FP32 sum), added in FP64.  FP32 D lane (i, q) register r
// = row 4 q + r, column i (the BF16 MFMA has the same output layout).
constexpr int kSKs = 32;  // reduction depth per stage

template <class T>
__device__ __forceinline__ void sk_load(const T* __restrict__ X, long long ld, long long rows, long long i0,
                                        long long k0, long long kend, T (&r)[16]) {
  // 128 x 32 tile, thread t: kk = t / 8, rows i0 + (t % 8) * 16 + e; loads
  // only (clamped addresses); sk_mask zeroes the out-of-range entries later
  const int t = threadIdx.x;
  const long long kk = k0 + t / 8;
  const long long ib = i0 + (t % 8) * 16;
  const T* p = X + (kk < kend ? kk : 0) * ld;
#pragma unroll
  for (int e = 0; e < 16; ++e) r[e] = p[ib + e < rows ? ib + e : 0];
}

__device__ __forceinline__ bool sk_in(long long rows, long long i0, long long k0, long long kend, int e) {
  const int t = threadIdx.x;
  return k0 + t / 8 < kend && i0 + (t % 8) * 16 + e < rows;
}

template <bool BF16>
__global__ void __launch_bounds__(kGThreads)
    k_sketch_gemm(const float* __restrict__ A, long long n, long long m, long long lda, const double* __restrict__ S,
                  long long srows, double* __restrict__ Y) {
  __shared__ float As[kSKs][kGM + 4];
  __shared__ float Bs[kSKs][kGM + 4];
  const long long i0 = (long long)blockIdx.x * kGM, j0 = (long long)blockIdx.y * kGM;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int li = lane % 16, lq = lane / 16;
  const int wr = wave / 2, wc = wave % 2;
  f64x4_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f64x4_t{0.0, 0.0, 0.0, 0.0};
  float ra[16];
  double rs[16];
  sk_load<float>(A, lda, n, i0, 0, m, ra);
  sk_load<double>(S, srows, srows, j0, 0, m, rs);
  for (long long k0 = 0; k0 < m; k0 += kSKs) {
    __syncthreads();
    {
      const int t = threadIdx.x, kk = t / 8, ib = (t % 8) * 16;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        As[kk][ib + e] = sk_in(n, i0, k0, m, e) ? ra[e] : 0.0f;
        Bs[kk][ib + e] = sk_in(srows, j0, k0, m, e) ? (float)rs[e] : 0.0f;
      }
    }
    __syncthreads();
    if (k0 + kSKs < m) {
      sk_load<float>(A, lda, n, i0, k0 + kSKs, m, ra);
      sk_load<double>(S, srows, srows, j0, k0 + kSKs, m, rs);
    }
    if (BF16) {
      bf16x8_t a[4], b[4];
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          a[t][e] = (__bf16)As[8 * lq + e][wr * 64 + t * 16 + li];
          b[t][e] = (__bf16)Bs[8 * lq + e][wc * 64 + t * 16 + li];
        }
#pragma unroll
      for (int ti = 0; ti < 4; ++ti)
#pragma unroll
        for (int tj = 0; tj < 4; ++tj) {
          f32x4_t c = {0.f, 0.f, 0.f, 0.f};
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ti], b[tj], c, 0, 0, 0);
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[ti][tj][r] += (double)c[r];
        }
    } else {
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        f32x4_t c[4][4];
#pragma unroll
        for (int ti = 0; ti < 4; ++ti)
#pragma unroll
          for (int tj = 0; tj < 4; ++tj) c[ti][tj] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = half * 16; kk < half * 16 + 16; kk += 4) {
          float a[4], b[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            a[t] = As[kk + lq][wr * 64 + t * 16 + li];
            b[t] = Bs[kk + lq][wc * 64 + t * 16 + li];
          }
#pragma unroll
          for (int ti = 0; ti < 4; ++ti)
#pragma unroll
            for (int tj = 0; tj < 4; ++tj)
              c[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ti], b[tj], c[ti][tj], 0, 0, 0);
        }
#pragma unroll
        for (int ti = 0; ti < 4; ++ti)
#pragma unroll
          for (int tj = 0; tj < 4; ++tj)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[ti][tj][r] += (double)c[ti][tj][r];
      }
    }
  }
  // D lane (i, q) register r = row 4 q + r, column i
#pragma unroll
  for (int ti = 0; ti < 4; ++ti)
#pragma unroll
    for (int tj = 0; tj < 4; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long long row = i0 + wr * 64 + ti * 16 + 4 * lq + r;  // column of A (output row of Y^T)
        const long long col = j0 + wc * 64 + tj * 16 + li;          // sketch row
        if (row < n && col < srows) Y[col * n + row] = acc[ti][tj][r];
      }
}

void sketch_gemm_f32(const float* A, long long m, long long n, long long lda, const double* S, int s_rows,
                     double* Y, bool bf16, hipStream_t st) {
  const dim3 g((unsigned)((n + kGM - 1) / kGM), (unsigned)((s_rows + kGM - 1) / kGM));
  if (bf16)
    hipLaunchKernelGGL(k_sketch_gemm<true>, g, dim3(kGThreads), 0, st, A, n, m, lda, S, (long long)s_rows, Y);
  else
    hipLaunchKernelGGL(k_sketch_gemm<false>, g, dim3(kGThreads), 0, st, A, n, m, lda, S, (long long)s_rows, Y);
}

}  // namespace aplicur
