// Blocked Golub-Kahan / LSQR kernels for several right-hand sides of a dense A
// (the recurrences of Sec. 2.2 per column, the products shared).
//
// Products.  A t, A^T u and the two products of the explicit P^{-1} are all
// "row-streaming" products out = M In with M row-major (A, its transposed
// copy, V^T or V) and In a row-major block of kp <= 64 columns.  They run on
// the 16x16x4 MFMA (FP64, or FP32 for FP32 blocks): a wave owns 32 rows of M
// and all kp columns, each step covers 32 entries of the reduction index, and
// lane (i, q) = (lane % 16, lane / 16) holds M[row i][j0 + 8q .. j0 + 8q + 7],
// loaded as one contiguous 32- or 64-byte piece, so a wave's load covers 16
// whole 128-byte lines of M.  The reduction index is split into S chunks
// (grid.y) when the rows alone give too few workgroups; the chunk partials are
// summed in order by the consuming kernel, which also does the element-wise
// LSQR work of the single-column kernels and the per-column reductions.
//
// Reductions.  As in the single-column kernels, a producing kernel writes one
// partial per workgroup and column, and every workgroup of the consumer sums
// them in a fixed order, so all workgroups hold bitwise-identical scalars;
// threads c < kp advance the state of column c.
#include <hip/hip_ext.h>

#include "blk.h"
#include "prof.h"

#include <cstdint>
#include <type_traits>

namespace aplicur {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <class ACC>
struct Mfma;
// row(q, r): the output row that register r of lane (i, q) holds (column i).
template <>
struct Mfma<double> {
  using acc_t = f64x4;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int q, int r) { return q + 4 * r; }
};
template <>
struct Mfma<float> {
  using acc_t = f32x4;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int q, int r) { return 4 * q + r; }
};

constexpr int kGT = 2;                               // 16-row tiles per wave
constexpr int kGRows = (kBlock / kWave) * kGT * 16;  // rows per workgroup
constexpr int kGPL = 8;                              // reduction entries per lane per step
constexpr int kGStep = 4 * kGPL;                     // reduction entries per step

// One step's operands: this lane's eight M values of each row tile (kept in
// M's type until the MFMA) and eight In values of each 16-column block.
template <class TA, class TB, int NB>
struct GemmStep {
  TA a[kGT][kGPL];
  TB b[NB][kGPL];
};

template <class TA, class TB, int NB, bool VEC>
__device__ __forceinline__ void gemm_load(GemmStep<TA, TB, NB>& st, const TA* const (&mrow)[kGT],
                                          const TB* __restrict__ In, long long j0, long long je, int li, int lq) {
  constexpr int KP = NB * 16;
  const long long jl = j0 + kGPL * lq;
  if (VEC && j0 + kGStep <= je) {
#pragma unroll
    for (int t = 0; t < kGT; ++t) {
      if constexpr (sizeof(TA) == 4) {
#pragma unroll
        for (int h = 0; h < kGPL / 4; ++h) {
          const f32x4 u = ((const f32x4*)(mrow[t] + jl))[h];
          st.a[t][4 * h] = u.x; st.a[t][4 * h + 1] = u.y; st.a[t][4 * h + 2] = u.z; st.a[t][4 * h + 3] = u.w;
        }
      } else {
#pragma unroll
        for (int h = 0; h < kGPL / 2; ++h) {
          const f64x2 u = ((const f64x2*)(mrow[t] + jl))[h];
          st.a[t][2 * h] = u.x; st.a[t][2 * h + 1] = u.y;
        }
      }
    }
#pragma unroll
    for (int e = 0; e < kGPL; ++e)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) st.b[nb][e] = In[(jl + e) * KP + nb * 16 + li];
  } else {
#pragma unroll
    for (int e = 0; e < kGPL; ++e) {
      const long long j = jl + e;
      const bool in = j < je;
      const long long jc = in ? j : je - 1;
#pragma unroll
      for (int t = 0; t < kGT; ++t) st.a[t][e] = in ? mrow[t][jc] : (TA)0;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) st.b[nb][e] = in ? In[jc * KP + nb * 16 + li] : (TB)0;
    }
  }
}

// MFMA 16x16x4 operands: A lane (i, q) holds row i, reduction entry q; B lane
// (i, q) holds entry q, column i; D lane (i, q) register r holds column i of
// row Mfma::row(q, r) (q + 4r for FP64: measured on gfx950; 4q + r for FP32).
// Here entry q of MFMA e is reduction index j0 + kGPL q + e.  The loads of step
// j + 1 are issued before the MFMAs of step j (two register stages).
template <class TA, class TB, class ACC, int NB, bool VEC>
__global__ void __launch_bounds__(kBlock)
    k_rows_gemm(const TA* __restrict__ M, long long rows, long long cols, long long ld, const TB* __restrict__ In,
                ACC* __restrict__ out, long long kchunk) {
  using MF = Mfma<ACC>;
  using acc_t = typename MF::acc_t;
  constexpr int KP = NB * 16;
  acc_t acc[kGT][NB];
#pragma unroll
  for (int t = 0; t < kGT; ++t)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[t][b] = acc_t{0, 0, 0, 0};
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int li = lane % 16, lq = lane / 16;
  const long long row0 = (long long)blockIdx.x * kGRows + (long long)wave * (kGT * 16);
  const long long jb = (long long)blockIdx.y * kchunk;
  const long long je = min(cols, jb + kchunk);
  const TA* mrow[kGT];
#pragma unroll
  for (int t = 0; t < kGT; ++t) mrow[t] = M + min(row0 + t * 16 + li, rows - 1) * ld;
  auto mma = [&](const GemmStep<TA, TB, NB>& st) {
#pragma unroll
    for (int e = 0; e < kGPL; ++e)
#pragma unroll
      for (int t = 0; t < kGT; ++t)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          acc[t][nb] = MF::op((ACC)st.a[t][e], (ACC)st.b[nb][e], acc[t][nb]);
  };
  if (jb < je) {
    GemmStep<TA, TB, NB> s0, s1;
    gemm_load<TA, TB, NB, VEC>(s0, mrow, In, jb, je, li, lq);
    for (long long j0 = jb;;) {
      const long long j1 = j0 + kGStep;
      if (j1 < je) gemm_load<TA, TB, NB, VEC>(s1, mrow, In, j1, je, li, lq);
      mma(s0);
      if (j1 >= je) break;
      const long long j2 = j1 + kGStep;
      if (j2 < je) gemm_load<TA, TB, NB, VEC>(s0, mrow, In, j2, je, li, lq);
      mma(s1);
      if (j2 >= je) break;
      j0 = j2;
    }
  }
  ACC* o = out + (long long)blockIdx.y * rows * KP;
#pragma unroll
  for (int t = 0; t < kGT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const long long row = row0 + t * 16 + MF::row(lq, r);
      if (row < rows) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) o[row * KP + nb * 16 + li] = acc[t][nb][r];
      }
    }
}

// The same product for FP64 In and 16 columns with FP64 accumulation (the
// several-RHS products of a dense A, and the blocked P-apply products), with
// In staged through LDS: the workgroup's four waves share one copy of each
// 128-entry chunk of In (16 KB, loaded with 16-byte loads by all threads
// during the previous chunk, double-buffered), so the L1 carries M once and
// In once per workgroup instead of once per wave.  M stays in registers (two
// stages), as above.  LDS rows of the chunk are 18 doubles apart, so the four
// 16-lane groups of a B-operand read fall on two bank halves.
constexpr int kXC = 4;               // steps per In chunk
constexpr int kXE = kXC * kGStep;    // entries per chunk
constexpr int kXLd = 18;             // LDS row stride of a chunk (doubles)

template <class TA>
struct AStep {
  TA a[kGT][kGPL];
};

template <class TA, bool VEC>
__device__ __forceinline__ void astep_load(AStep<TA>& st, const TA* const (&mrow)[kGT], long long j0, long long je,
                                           int lq) {
  const long long jl = j0 + kGPL * lq;
  if (VEC && j0 + kGStep <= je) {
#pragma unroll
    for (int t = 0; t < kGT; ++t) {
      if constexpr (sizeof(TA) == 4) {
#pragma unroll
        for (int h = 0; h < kGPL / 4; ++h) {
          const f32x4 u = ((const f32x4*)(mrow[t] + jl))[h];
          st.a[t][4 * h] = u.x; st.a[t][4 * h + 1] = u.y; st.a[t][4 * h + 2] = u.z; st.a[t][4 * h + 3] = u.w;
        }
      } else {
#pragma unroll
        for (int h = 0; h < kGPL / 2; ++h) {
          const f64x2 u = ((const f64x2*)(mrow[t] + jl))[h];
          st.a[t][2 * h] = u.x; st.a[t][2 * h + 1] = u.y;
        }
      }
    }
  } else {
#pragma unroll
    for (int e = 0; e < kGPL; ++e) {
      const long long j = jl + e;
      const bool in = j < je;
      const long long jc = in ? j : je - 1;
#pragma unroll
      for (int t = 0; t < kGT; ++t) st.a[t][e] = in ? mrow[t][jc] : (TA)0;
    }
  }
}

template <class TA, bool VEC>
__global__ void __launch_bounds__(kBlock)
    k_rows_gemm_xl(const TA* __restrict__ M, long long rows, long long cols, long long ld,
                   const double* __restrict__ In, double* __restrict__ out, long long kchunk) {
  constexpr int KP = 16;
  constexpr int NX = kXE * KP / 2 / kBlock;  // 16-byte loads of a chunk per thread
  __shared__ double Xs[2][kXE][kXLd];
  f64x4 acc[kGT];
#pragma unroll
  for (int t = 0; t < kGT; ++t) acc[t] = f64x4{0, 0, 0, 0};
  const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
  const int li = lane % 16, lq = lane / 16;
  const long long row0 = (long long)blockIdx.x * kGRows + (long long)wave * (kGT * 16);
  const long long jb = (long long)blockIdx.y * kchunk;
  const long long je = min(cols, jb + kchunk);
  const TA* mrow[kGT];
#pragma unroll
  for (int t = 0; t < kGT; ++t) mrow[t] = M + min(row0 + t * 16 + li, rows - 1) * ld;
  auto xload = [&](long long c0, f64x2 (&r)[NX]) {
#pragma unroll
    for (int k = 0; k < NX; ++k) {
      const int idx = tid + k * kBlock;
      const long long j = c0 + idx / (KP / 2);
      r[k] = j < je ? ((const f64x2*)(In + j * KP))[idx % (KP / 2)] : f64x2{0.0, 0.0};
    }
  };
  auto xstore = [&](int buf, const f64x2 (&r)[NX]) {
#pragma unroll
    for (int k = 0; k < NX; ++k) {
      const int idx = tid + k * kBlock;
      *(f64x2*)&Xs[buf][idx / (KP / 2)][2 * (idx % (KP / 2))] = r[k];
    }
  };
  auto mma = [&](const AStep<TA>& st, int buf, int s) {
#pragma unroll
    for (int e = 0; e < kGPL; ++e) {
      const double bv = Xs[buf][s * kGStep + kGPL * lq + e][li];
#pragma unroll
      for (int t = 0; t < kGT; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)st.a[t][e], bv, acc[t], 0, 0, 0);
    }
  };
  if (jb < je) {  // uniform
    f64x2 xr[NX];
    xload(jb, xr);
    xstore(0, xr);
    __syncthreads();
    AStep<TA> s0, s1;
    astep_load<TA, VEC>(s0, mrow, jb, je, lq);
    int buf = 0;
    for (long long c0 = jb; c0 < je; c0 += kXE) {
      const long long c1 = c0 + kXE;
      if (c1 < je) xload(c1, xr);  // in flight during this chunk's steps
      // kXC is even, so every chunk starts with its first step in s0
#pragma unroll
      for (int s = 0; s < kXC; s += 2) {
        const long long j0 = c0 + s * kGStep, j1 = j0 + kGStep, j2 = j1 + kGStep;
        if (j0 >= je) break;
        if (j1 < je) astep_load<TA, VEC>(s1, mrow, j1, je, lq);
        mma(s0, buf, s);
        if (j1 >= je) break;
        if (j2 < je) astep_load<TA, VEC>(s0, mrow, j2, je, lq);
        mma(s1, buf, s + 1);
      }
      if (c1 < je) xstore(buf ^ 1, xr);
      __syncthreads();
      buf ^= 1;
    }
  }
  double* o = out + (long long)blockIdx.y * rows * KP;
#pragma unroll
  for (int t = 0; t < kGT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const long long row = row0 + t * 16 + lq + 4 * r;
      if (row < rows) o[row * KP + li] = acc[t][r];
    }
}

int gemm_splits(long long rows, long long cols) {
  const long long gx = ceil_div(rows, kGRows);
  long long S = (1024 + gx - 1) / gx;  // about four workgroups per CU
  S = std::min<long long>(S, std::max<long long>(1, cols / 512));
  return (int)std::max<long long>(1, std::min<long long>(S, 64));
}

// Launch; with events, through the dispatch-timed launch (the events take
// the kernel's own start and end timestamps).
template <class F, class... Args>
static void launch_ev(F kern, dim3 g, hipStream_t s, hipEvent_t e0, hipEvent_t e1, Args... args) {
  if (e0 || e1)
    hipExtLaunchKernelGGL(kern, g, dim3(kBlock), 0, s, e0, e1, 0, args...);
  else
    hipLaunchKernelGGL(kern, g, dim3(kBlock), 0, s, args...);
}

template <class TA, class TB, class ACC, int NB>
static void rows_gemm_nb(const TA* M, long long rows, long long cols, long long ld, const TB* In, ACC* out, int S,
                         hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const long long per = ceil_div(cols, S);
  const long long kchunk = ((per + kGStep - 1) / kGStep) * kGStep;
  const bool vec = ((uintptr_t)M % 16 == 0) && ((ld * (long long)sizeof(TA)) % 16 == 0);
  const dim3 g(ceil_div(rows, kGRows), S);
  if constexpr (std::is_same<TB, double>::value && std::is_same<ACC, double>::value && NB == 1) {
    // FP64 In, 16 columns, FP64 accumulation: In staged in LDS once per workgroup
    if (vec)
      launch_ev(k_rows_gemm_xl<TA, true>, g, s, e0, e1, M, rows, cols, ld, In, out, kchunk);
    else
      launch_ev(k_rows_gemm_xl<TA, false>, g, s, e0, e1, M, rows, cols, ld, In, out, kchunk);
    return;
  }
  if (vec)
    launch_ev(k_rows_gemm<TA, TB, ACC, NB, true>, g, s, e0, e1, M, rows, cols, ld, In, out, kchunk);
  else
    launch_ev(k_rows_gemm<TA, TB, ACC, NB, false>, g, s, e0, e1, M, rows, cols, ld, In, out, kchunk);
}

template <class TA, class TB, class ACC>
void rows_gemm(const TA* M, long long rows, long long cols, long long ld, const TB* In, int kp, ACC* out, int S,
               hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  APL_REQUIRE(rows >= 1 && cols >= 1 && S >= 1, "rows_gemm: empty product");
  switch (kp) {
    case 16: rows_gemm_nb<TA, TB, ACC, 1>(M, rows, cols, ld, In, out, S, s, e0, e1); break;
    case 32: rows_gemm_nb<TA, TB, ACC, 2>(M, rows, cols, ld, In, out, S, s, e0, e1); break;
    case 64: rows_gemm_nb<TA, TB, ACC, 4>(M, rows, cols, ld, In, out, S, s, e0, e1); break;
    default: APL_REQUIRE(false, "rows_gemm: kp must be 16, 32 or 64");
  }
}
template void rows_gemm<double, double, double>(const double*, long long, long long, long long, const double*, int,
                                                double*, int, hipStream_t, hipEvent_t, hipEvent_t);
template void rows_gemm<float, double, double>(const float*, long long, long long, long long, const double*, int,
                                               double*, int, hipStream_t, hipEvent_t, hipEvent_t);
template void rows_gemm<float, float, float>(const float*, long long, long long, long long, const float*, int, float*,
                                             int, hipStream_t, hipEvent_t, hipEvent_t);
template void rows_gemm<double, float, double>(const double*, long long, long long, long long, const float*, int,
                                               double*, int, hipStream_t, hipEvent_t, hipEvent_t);

// ---------------------------------------------------------------- layout helpers
template <class T>
__global__ void __launch_bounds__(kBlock)
    k_transpose_rect(const T* __restrict__ A, long long m, long long n, long long lda, T* __restrict__ At,
                     long long ldt) {
  __shared__ T tile[32][33];
  const long long i0 = (long long)blockIdx.y * 32, j0 = (long long)blockIdx.x * 32;
  const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
  for (int r = ty; r < 32; r += kBlock / 32) {
    const long long i = i0 + r, j = j0 + tx;
    if (i < m && j < n) tile[r][tx] = A[i * lda + j];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += kBlock / 32) {
    const long long j = j0 + r, i = i0 + tx;
    if (j < n && i < m) At[j * ldt + i] = tile[tx][r];
  }
}

template <class T>
void transpose_rect(const T* A, long long m, long long n, long long lda, T* At, long long ldt, hipStream_t s) {
  APL_REQUIRE(ceil_div(m, 32) <= 65535, "transpose_rect: too many rows");
  hipLaunchKernelGGL((k_transpose_rect<T>), dim3(ceil_div(n, 32), ceil_div(m, 32)), dim3(kBlock), 0, s, A, m, n, lda,
                     At, ldt);
}
template void transpose_rect<double>(const double*, long long, long long, long long, double*, long long, hipStream_t);
template void transpose_rect<float>(const float*, long long, long long, long long, float*, long long, hipStream_t);

template <class TO>
__global__ void k_pack_cols(const double* __restrict__ X, long long ldx, long long rows, int k, TO* __restrict__ Xp,
                            int kp) {
  const long long total = rows * kp;
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < total; e += (long long)gridDim.x * kBlock) {
    const long long r = e / kp;
    const int c = (int)(e % kp);
    Xp[e] = c < k ? (TO)X[(long long)c * ldx + r] : (TO)0;
  }
}

__global__ void k_unpack_cols(const double* __restrict__ Xp, int kp, long long rows, int k, double* __restrict__ X,
                              long long ldx) {
  const long long total = rows * k;
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < total; e += (long long)gridDim.x * kBlock) {
    const int c = (int)(e / rows);
    const long long r = e % rows;
    X[(long long)c * ldx + r] = Xp[r * kp + c];
  }
}

// Y[:, c] = sum (in order, in TP) of the S planes of part (rows x kp) at column c, for c < k.
template <class TP>
__global__ void k_planes_to_cols(const TP* __restrict__ part, int S, long long rows, int kp, int k,
                                 double* __restrict__ Y, long long ldy) {
  const long long total = rows * k, plane = rows * kp;
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < total; e += (long long)gridDim.x * kBlock) {
    const int c = (int)(e / rows);
    const long long r = e % rows;
    TP acc = part[r * kp + c];
    for (int q = 1; q < S; ++q) acc += part[(long long)q * plane + r * kp + c];
    Y[(long long)c * ldy + r] = (double)acc;
  }
}

static unsigned elem_grid(long long count, long long cap = 4096) {
  long long g = ceil_div(count, kBlock);
  if (g < 1) g = 1;
  return (unsigned)(g > cap ? cap : g);
}

// ---------------------------------------------------------------- BF16 products
// BF16 copy of a row-major FP32 matrix in tiles of 32 rows x 64 columns:
// element (r, j) at ((r / 32) NJ + j / 64) 2048 + (r % 32) 64 + j % 64 with
// NJ = ceil(cols / 64), rows and columns padded with zeros, so that one step
// of a wave in k_rows_gemm16 reads 4 KB of contiguous memory.  Values are
// rounded to nearest even.  Thread g writes 8 consecutive entries of a tile
// row (16 bytes) from 8 consecutive entries of the source row.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__global__ void __launch_bounds__(kBlock)
    k_tile_bf16(const float* __restrict__ src, long long rows, long long cols, long long ld, long long NJ,
                long long groups, __bf16* __restrict__ dst) {
  for (long long g = (long long)blockIdx.x * kBlock + threadIdx.x; g < groups; g += (long long)gridDim.x * kBlock) {
    const long long t = g / 256, w = g % 256;
    const long long r = (t / NJ) * 32 + w / 8, j0 = (t % NJ) * 64 + (w % 8) * 8;
    bf16x8 o;
#pragma unroll
    for (int e = 0; e < 8; ++e) o[e] = (__bf16)((r < rows && j0 + e < cols) ? src[r * ld + j0 + e] : 0.0f);
    *(bf16x8*)(dst + g * 8) = o;
  }
}

long long bf16_tiled_elems(long long rows, long long cols) { return (rows + 31) / 32 * 32 * ((cols + 63) / 64 * 64); }

void tile_bf16(const float* src, long long rows, long long cols, long long ld, void* dst, hipStream_t s) {
  const long long groups = bf16_tiled_elems(rows, cols) / 8;
  hipLaunchKernelGGL(k_tile_bf16, dim3(elem_grid(groups)), dim3(kBlock), 0, s, src, rows, cols, ld,
                     (cols + 63) / 64, groups, (__bf16*)dst);
}

// out[s] = (the s-th chunk of the reduction index of) T In for a tiled BF16
// T (rows x cols) and FP32 In (cols x KP row-major), FP32 accumulation, on
// the 16x16x32 BF16 MFMA: A lane (i, q) holds row i, entries 8q .. 8q + 7 of
// the 32; B lane (i, q) holds column i, the same entries; D lane (i, q)
// register r holds row 4q + r, column i (the FP32 16x16x4 layout; checked on
// gfx950).  Lane (i, q) loads T[row i][j0 + GPL q .. + GPL) (16 or 32
// contiguous bytes) and sub-step h < GPL / 8 feeds entries GPL q + 8h + e
// (e < 8) to one MFMA: a permutation of the reduction index.  In is split
// into BF16 hi + lo parts (two MFMAs), so the product carries the rounding of
// T and In's to about 2^-16 only.  Steps have 4 GPL entries; chunk bounds
// are multiples of 64, and only In needs guarding in a step that crosses
// cols (T is zero-padded to whole tiles).  Two register stages as in
// k_rows_gemm.
template <int NB, int GPL>
struct Gemm16Step {
  bf16x8 a[kGT][GPL / 8];
  float b[NB][GPL];
};

template <int NB, int GPL>
__global__ void __launch_bounds__(kBlock)
    k_rows_gemm16(const __bf16* __restrict__ T, long long rows, long long cols, long long NJ,
                  const float* __restrict__ In, float* __restrict__ out, long long kchunk) {
  constexpr int KP = NB * 16, ST = 4 * GPL;
  f32x4 acc[kGT][NB];
#pragma unroll
  for (int t = 0; t < kGT; ++t)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[t][b] = f32x4{0, 0, 0, 0};
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int li = lane % 16, lq = lane / 16;
  const long long row0 = (long long)blockIdx.x * kGRows + (long long)wave * (kGT * 16);
  const long long jb = (long long)blockIdx.y * kchunk;
  const long long je = min(cols, jb + kchunk);
  const long long R = min(row0 / 32, (rows + 31) / 32 - 1);  // waves past the last tile read it and store nothing
  const __bf16* base[kGT];
#pragma unroll
  for (int t = 0; t < kGT; ++t) base[t] = T + R * NJ * 2048 + (16 * t + li) * 64 + GPL * lq;
  auto load = [&](Gemm16Step<NB, GPL>& st, long long j0) {
    const long long off = (j0 / 64) * 2048 + j0 % 64;
#pragma unroll
    for (int t = 0; t < kGT; ++t)
#pragma unroll
      for (int h = 0; h < GPL / 8; ++h) st.a[t][h] = *((const bf16x8*)(base[t] + off) + h);
    const long long jl = j0 + GPL * lq;
    if (j0 + ST <= je) {
#pragma unroll
      for (int e = 0; e < GPL; ++e)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) st.b[nb][e] = In[(jl + e) * KP + nb * 16 + li];
    } else {
#pragma unroll
      for (int e = 0; e < GPL; ++e) {
        const bool in = jl + e < je;
        const long long jc = in ? jl + e : je - 1;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const float v = In[jc * KP + nb * 16 + li];
          st.b[nb][e] = in ? v : 0.0f;
        }
      }
    }
  };
  auto mma = [&](const Gemm16Step<NB, GPL>& st) {
#pragma unroll
    for (int h = 0; h < GPL / 8; ++h)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        bf16x8 hi, lo;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float x = st.b[nb][8 * h + e];
          hi[e] = (__bf16)x;
          lo[e] = (__bf16)(x - (float)hi[e]);
        }
#pragma unroll
        for (int t = 0; t < kGT; ++t) {
          acc[t][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(st.a[t][h], hi, acc[t][nb], 0, 0, 0);
          acc[t][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(st.a[t][h], lo, acc[t][nb], 0, 0, 0);
        }
      }
  };
  if (jb < je) {
    Gemm16Step<NB, GPL> s0, s1;
    load(s0, jb);
    for (long long j0 = jb;;) {
      const long long j1 = j0 + ST;
      if (j1 < je) load(s1, j1);
      mma(s0);
      if (j1 >= je) break;
      const long long j2 = j1 + ST;
      if (j2 < je) load(s0, j2);
      mma(s1);
      if (j2 >= je) break;
      j0 = j2;
    }
  }
  float* o = out + (long long)blockIdx.y * rows * KP;
#pragma unroll
  for (int t = 0; t < kGT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const long long row = row0 + t * 16 + 4 * lq + r;
      if (row < rows) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) o[row * KP + nb * 16 + li] = acc[t][nb][r];
      }
    }
}

void rows_gemm16(const void* T, long long rows, long long cols, const float* In, int kp, float* out, int S,
                 hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  APL_REQUIRE(rows >= 1 && cols >= 1 && S >= 1, "rows_gemm16: empty product");
  const long long kchunk = ((cols + S - 1) / S + 63) / 64 * 64;
  const dim3 g((unsigned)ceil_div(rows, kGRows), (unsigned)S);
  const long long NJ = (cols + 63) / 64;
  const __bf16* M = (const __bf16*)T;
  switch (kp) {
    case 16:
      launch_ev(k_rows_gemm16<1, 16>, g, s, e0, e1, M, rows, cols, NJ, In, out, kchunk);
      break;
    case 32:
      launch_ev(k_rows_gemm16<2, 16>, g, s, e0, e1, M, rows, cols, NJ, In, out, kchunk);
      break;
    case 64:
      launch_ev(k_rows_gemm16<4, 8>, g, s, e0, e1, M, rows, cols, NJ, In, out, kchunk);
      break;
    default: APL_REQUIRE(false, "rows_gemm16: kp must be 16, 32 or 64");
  }
}


void pack_cols(const double* X, long long ldx, long long rows, int k, double* Xp, int kp, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_cols<double>, dim3(elem_grid(rows * kp)), dim3(kBlock), 0, s, X, ldx, rows, k, Xp, kp);
}
void unpack_cols(const double* Xp, int kp, long long rows, int k, double* X, long long ldx, hipStream_t s) {
  hipLaunchKernelGGL(k_unpack_cols, dim3(elem_grid(rows * k)), dim3(kBlock), 0, s, Xp, kp, rows, k, X, ldx);
}

void blk_matmat(const BlkOp& A, bool trans, const double* X, long long ldx, int kp, int k, double* Y, long long ldy,
                int prec, void* in, void* part, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const long long rows = trans ? A.n : A.m, cols = trans ? A.m : A.n, ld = trans ? A.ldt : A.ld;
  const void* M = trans ? A.At : A.A;
  const int S = trans ? A.Sn : A.Sm;
  const unsigned gi = elem_grid(cols * kp), go = elem_grid(rows * k);
  if (prec == 0) {
    hipLaunchKernelGGL(k_pack_cols<double>, dim3(gi), dim3(kBlock), 0, s, X, ldx, cols, k, (double*)in, kp);
    if (A.f64)
      rows_gemm<double, double, double>((const double*)M, rows, cols, ld, (const double*)in, kp, (double*)part, S, s,
                                        e0, e1);
    else
      rows_gemm<float, double, double>((const float*)M, rows, cols, ld, (const double*)in, kp, (double*)part, S, s,
                                       e0, e1);
    hipLaunchKernelGGL(k_planes_to_cols<double>, dim3(go), dim3(kBlock), 0, s, (const double*)part, S, rows, kp, k, Y,
                       ldy);
    return;
  }
  APL_REQUIRE(!A.f64 && (prec == 1 || A.A16), "blk_matmat: no FP32 / BF16 operator");
  hipLaunchKernelGGL(k_pack_cols<float>, dim3(gi), dim3(kBlock), 0, s, X, ldx, cols, k, (float*)in, kp);
  if (prec == 1)
    rows_gemm<float, float, float>((const float*)M, rows, cols, ld, (const float*)in, kp, (float*)part, S, s, e0, e1);
  else
    rows_gemm16(trans ? A.At16 : A.A16, rows, cols, (const float*)in, kp, (float*)part, S, s, e0, e1);
  hipLaunchKernelGGL(k_planes_to_cols<float>, dim3(go), dim3(kBlock), 0, s, (const float*)part, S, rows, kp, k, Y, ldy);
}

// ---------------------------------------------------------------- per-column reductions
// out[c] = sum over w < count of part[w kp + c], in a fixed order (thread
// c + kp q takes w = q, q + NS, ...; then q in order).  All threads call.
template <int KP>
__device__ __forceinline__ void col_sums(const double* __restrict__ part, int count, double* lds, double* out) {
  constexpr int NS = kBlock / KP;
  const int c = threadIdx.x % KP, q = threadIdx.x / KP;
  double acc = 0.0;
  if (part) {
#pragma unroll 4
    for (int w = q; w < count; w += NS) acc += part[(long long)w * KP + c];
  }
  lds[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x < KP) {
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < NS; ++i) t += lds[i * KP + threadIdx.x];
    out[threadIdx.x] = t;
  }
  __syncthreads();
}

// This workgroup's partial of column (threadIdx.x % kp): part_out[blockIdx.x kp + c].
template <int KP>
__device__ __forceinline__ void col_partials(double sq, double* lds, double* part_out) {
  constexpr int NS = kBlock / KP;
  __syncthreads();
  lds[threadIdx.x] = sq;
  __syncthreads();
  if (threadIdx.x < KP) {
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < NS; ++i) t += lds[i * KP + threadIdx.x];
    part_out[(long long)blockIdx.x * KP + threadIdx.x] = t;
  }
}

// Sum of the S chunk planes of a product at element e.
template <class V>
__device__ __forceinline__ V plane_sum(const V* __restrict__ part, int S, long long plane, long long e) {
  V acc = part[e];
  for (int s = 1; s < S; ++s) acc += part[(long long)s * plane + e];
  return acc;
}

// Per-column scalars shared through LDS.
struct BlkScal {
  double ts, cu, cy, cw, ib, cv;
  int active, pend, fin, init;
};

// ---------------------------------------------------------------- phase start
// r_top = B - (A X) (FP64 partials; B when pm is null), r_bot = bs Bbot - delta X;
// partials of ||r||^2 per column.
template <class RV, int KP>
__global__ void __launch_bounds__(kBlock)
    k_blk_resid(const double* __restrict__ pm, int S, long long m, long long n, const double* __restrict__ B,
                const double* Bbot, double bs, const double* X, double delta, RV* r_top, RV* r_bot,
                double* beta_part) {
  __shared__ double lds[kBlock];
  const long long stride = (long long)gridDim.x * kBlock;
  double sq = 0.0;
  const long long mp = m * KP, np = n * KP;
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < mp; e += stride) {
    const double r = (B ? B[e] : 0.0) - (pm ? plane_sum(pm, S, mp, e) : 0.0);
    r_top[e] = (RV)r;
    sq += r * r;
  }
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < np; e += stride) {
    double r = X ? -delta * X[e] : 0.0;
    if (Bbot) r += bs * Bbot[e];
    r_bot[e] = (RV)r;
    sq += r * r;
  }
  col_partials<KP>(sq, lds, beta_part);
}

// ---------------------------------------------------------------- forward
// u_top <- (A tin) / alpha - (alpha / beta) u_top, u_bot likewise, partials of
// ||u||^2.  PLAIN finishes alpha (slot 1 -> slot 0), takes the scalar step and
// applies the previous y/w update; PRE uses slot 0 as the P^{-1} kernel left it.
template <class V, int KP, int MODE>
__global__ void __launch_bounds__(kBlock)
    k_blk_fwd(const V* __restrict__ pm, int S, long long m, long long n, double delta, const V* tin, V* u_top,
              V* u_bot, const V* v, V* w, V* y, const GKState* __restrict__ st_in, GKState* __restrict__ st_out,
              const double* alpha_part, int alpha_count, double* beta_part) {
  __shared__ double lds[kBlock];
  __shared__ double a2[KP];
  __shared__ BlkScal sc[KP];
  if (MODE == kFwdPlain) col_sums<KP>(alpha_part, alpha_count, lds, a2);
  if (threadIdx.x < KP) {
    const int c = threadIdx.x;
    GKState s = st_in[c];
    BlkScal k{};
    if (!s.stop) {
      if (MODE == kFwdPlain) scalar_step(s, sqrt(a2[c]));
      if (s.stop) {
        k.fin = s.pending;
        k.cy = s.coef_y;
      } else {
        k.active = 1;
        k.ts = 1.0 / s.alpha;
        k.cu = s.alpha / s.beta;
        k.pend = (MODE == kFwdPlain) && s.pending;
        k.cy = s.coef_y;
        k.cw = s.coef_w;
      }
    }
    if (MODE == kFwdPlain && blockIdx.x == 0) st_out[c] = s;
    sc[c] = k;
  }
  __syncthreads();
  const BlkScal k = sc[threadIdx.x % KP];
  const V ts = (V)k.ts, cu = (V)k.cu, cy = (V)k.cy, cw = (V)k.cw;
  const long long stride = (long long)gridDim.x * kBlock;
  double sq = 0.0;
  if (k.active) {
    const long long mp = m * KP;
    for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < mp; e += stride) {
      const V un = plane_sum(pm, S, mp, e) * ts - cu * u_top[e];
      u_top[e] = un;
      sq += (double)un * (double)un;
    }
  }
  if (k.active || k.fin) {
    const long long np = n * KP;
    for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < np; e += stride) {
      if (k.active) {
        if (delta > 0.0) {
          const V ub = (V)delta * (tin[e] * ts) - cu * u_bot[e];
          u_bot[e] = ub;
          sq += (double)ub * (double)ub;
        }
        if (k.pend) {
          const V we = w[e];
          y[e] += cy * we;
          w[e] = v[e] * ts - cw * we;
        }
      } else {
        y[e] += cy * w[e];
      }
    }
  }
  col_partials<KP>(sq, lds, beta_part);
}

// ---------------------------------------------------------------- backward
// beta from the forward partials (slot 0 -> slot 1); g = (A^T u_top + delta
// u_bot) / beta.  PLAIN: v <- g - (beta / alpha) v (g at the phase start) and
// partials of ||v||^2; otherwise g is stored for P^{-T}.
template <class V, int KP, bool PLAIN>
__global__ void __launch_bounds__(kBlock)
    k_blk_bwd(const V* __restrict__ pn, int S, long long n, double delta, const V* u_bot, V* v, V* g,
              const GKState* __restrict__ st_in, GKState* __restrict__ st_out, const double* beta_part, int beta_count,
              double* alpha_part) {
  __shared__ double lds[kBlock];
  __shared__ double b2[KP];
  __shared__ BlkScal sc[KP];
  col_sums<KP>(beta_part, beta_count, lds, b2);
  if (threadIdx.x < KP) {
    const int c = threadIdx.x;
    GKState s = st_in[c];
    BlkScal k{};
    if (!s.stop) {
      const double beta = sqrt(b2[c]);
      const bool bad = !(beta == beta) || isinf(beta) || (beta == 0.0 && s.init);
      const double alpha = s.alpha;
      k.init = s.init;
      beta_step(s, b2[c]);
      if (!bad && beta != 0.0) {
        k.active = 1;
        k.ib = 1.0 / beta;
        k.cv = beta / alpha;
      }
    }
    if (blockIdx.x == 0) st_out[c] = s;
    sc[c] = k;
  }
  __syncthreads();
  const BlkScal k = sc[threadIdx.x % KP];
  const V ib = (V)k.ib, cv = (V)k.cv;
  double sq = 0.0;
  if (k.active) {
    const long long np = n * KP;
    for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < np; e += (long long)gridDim.x * kBlock) {
      V ge = plane_sum(pn, S, np, e) * ib;
      if (delta > 0.0) ge += (V)delta * u_bot[e] * ib;
      if (PLAIN) {
        const V vn = k.init ? ge : ge - cv * v[e];
        v[e] = vn;
        sq += (double)vn * (double)vn;
      } else {
        g[e] = ge;
      }
    }
  }
  if (PLAIN) col_partials<KP>(sq, lds, alpha_part);
}

// ---------------------------------------------------------------- explicit P^{-1}
// c = d .* (sum of the S planes of V^T z), ell x kp (d null: the plain sum).
template <int KP>
__global__ void __launch_bounds__(kBlock)
    k_blk_pcoef(const double* __restrict__ pl, int S, int ell, const double* __restrict__ d, double* c) {
  const long long lp = (long long)ell * KP;
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < lp; e += (long long)gridDim.x * kBlock)
    c[e] = d ? d[e / KP] * plane_sum(pl, S, lp, e) : plane_sum(pl, S, lp, e);
}

// First kernel of a preconditioned iteration: alpha (slot 1 -> slot 0), the
// scalar step, the y/w update and t = v + V c.
template <class V, int KP>
__global__ void __launch_bounds__(kBlock)
    k_blk_pa_fwd(const double* __restrict__ pq, int S, long long n, const V* v, V* t, V* w, V* y,
                 const GKState* __restrict__ st_in, GKState* __restrict__ st_out, const double* alpha_part,
                 int alpha_count) {
  __shared__ double lds[kBlock];
  __shared__ double a2[KP];
  __shared__ BlkScal sc[KP];
  col_sums<KP>(alpha_part, alpha_count, lds, a2);
  if (threadIdx.x < KP) {
    const int c = threadIdx.x;
    GKState s = st_in[c];
    BlkScal k{};
    if (!s.stop) {
      scalar_step(s, sqrt(a2[c]));
      if (s.stop) {
        k.fin = s.pending;
        k.cy = s.coef_y;
      } else {
        k.active = 1;
        k.pend = s.pending;
        k.cy = s.coef_y;
        k.cw = s.coef_w;
        k.ts = 1.0 / s.alpha;
      }
    }
    if (blockIdx.x == 0) st_out[c] = s;
    sc[c] = k;
  }
  __syncthreads();
  const BlkScal k = sc[threadIdx.x % KP];
  if (!k.active && !k.fin) return;
  const long long np = n * KP;
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < np; e += (long long)gridDim.x * kBlock) {
    if (k.active) {
      const V ve = v[e];
      t[e] = (V)((double)ve + plane_sum(pq, S, np, e));
      if (k.pend) {
        const V we = w[e];
        y[e] += (V)k.cy * we;
        w[e] = (V)((double)ve * k.ts) - (V)k.cw * we;
      }
    } else {
      y[e] += (V)k.cy * w[e];
    }
  }
}

// v <- (g + V c) - (beta / alpha) v  (g + V c at the phase start); partials of
// ||v||^2 (slot 1 holds beta).
template <class V, int KP>
__global__ void __launch_bounds__(kBlock)
    k_blk_pa_bwd(const double* __restrict__ pq, int S, long long n, const V* g, V* v, const GKState* __restrict__ sl,
                 double* alpha_part) {
  __shared__ double lds[kBlock];
  __shared__ BlkScal sc[KP];
  if (threadIdx.x < KP) {
    const GKState& s = sl[threadIdx.x];
    BlkScal k{};
    if (!s.stop) {
      k.active = 1;
      k.init = s.init;
      k.cv = s.beta / s.alpha;
    }
    sc[threadIdx.x] = k;
  }
  __syncthreads();
  const BlkScal k = sc[threadIdx.x % KP];
  double sq = 0.0;
  if (k.active) {
    const long long np = n * KP;
    for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < np; e += (long long)gridDim.x * kBlock) {
      const double pg = (double)g[e] + plane_sum(pq, S, np, e);
      const V vn = k.init ? (V)pg : (V)(pg - k.cv * (double)v[e]);
      v[e] = vn;
      sq += (double)vn * (double)vn;
    }
  }
  col_partials<KP>(sq, lds, alpha_part);
}

// X += y (+ V c when pq is given), FP64.
template <class V>
__global__ void __launch_bounds__(kBlock)
    k_blk_add_x(const double* __restrict__ pq, int S, long long count, const V* __restrict__ y, double* X) {
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < count; e += (long long)gridDim.x * kBlock)
    X[e] += (double)y[e] + (pq ? plane_sum(pq, S, count, e) : 0.0);
}

// ---------------------------------------------------------------- norms
// Column partials of ||a||^2 over rows x kp (a given), or of
// ||plane sum of pn + delta r_bot||^2 (the normal residual) when pn is given;
// outv (optional) receives the summed vector.
template <int KP>
__global__ void __launch_bounds__(kBlock)
    k_blk_colsq(const double* __restrict__ a, const double* __restrict__ pn, int S, long long rows, double delta,
                const double* __restrict__ r_bot, double* part, double* outv) {
  __shared__ double lds[kBlock];
  const long long np = rows * KP;
  double sq = 0.0;
  for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < np; e += (long long)gridDim.x * kBlock) {
    double x;
    if (pn) {
      x = plane_sum(pn, S, np, e);
      if (r_bot) x += delta * r_bot[e];
    } else {
      x = a[e];
    }
    if (outv) outv[e] = x;
    sq += x * x;
  }
  col_partials<KP>(sq, lds, part);
}

// ---------------------------------------------------------------- host launchers
#define BLK_KP_SWITCH(kp, CALL)                            \
  switch (kp) {                                            \
    case 16: { constexpr int KP = 16; CALL; } break;       \
    case 32: { constexpr int KP = 32; CALL; } break;       \
    case 64: { constexpr int KP = 64; CALL; } break;       \
    default: APL_REQUIRE(false, "blocked path: kp must be 16, 32 or 64"); \
  }

static unsigned blk_grid(long long rows, int kp) { return elem_grid(rows * kp, kBlkMaxGrid); }

// A t (tin: n x kp) into the partials pm (Sm planes), or A^T u into pn.
template <class V>
static void blk_prod(const BlkOp& A, bool trans, const V* in, int kp, V* out, hipStream_t s) {
  const long long rows = trans ? A.n : A.m, cols = trans ? A.m : A.n, ld = trans ? A.ldt : A.ld;
  const void* M = trans ? A.At : A.A;
  const int S = trans ? A.Sn : A.Sm;
  constexpr bool f32 = std::is_same<V, float>::value;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  prof_take((trans ? 1 : 0) + (f32 ? (A.A16 ? 4 : 2) : 0), &e0, &e1);
  if constexpr (f32) {
    if (A.A16) {
      rows_gemm16(trans ? A.At16 : A.A16, rows, cols, in, kp, out, S, s, e0, e1);
      return;
    }
  }
  if (A.f64)
    rows_gemm<double, V, V>((const double*)M, rows, cols, ld, in, kp, out, S, s, e0, e1);
  else
    rows_gemm<float, V, V>((const float*)M, rows, cols, ld, in, kp, out, S, s, e0, e1);
}

// c = d .* V^T z, then pq = V c (S2 planes); in factored form c = W (Q_R^T z)
// and pq = Q_R c.
template <class V>
static void blk_pcoef(const BlkOp& A, const BlkPrec& P, int kp, const V* z, BlkWork& wk, hipStream_t s) {
  auto coef = [&](int S, const double* d, double* out) {
    BLK_KP_SWITCH(kp, hipLaunchKernelGGL((k_blk_pcoef<KP>), dim3(blk_grid(P.ell, kp)), dim3(kBlock), 0, s, wk.pl, S,
                                         P.ell, d, out));
  };
  rows_gemm<double, V, double>(P.Vt, P.ell, A.n, P.ldvt, z, kp, wk.pl, P.S1, s);
  double* c = wk.pc;
  if (P.W) {
    coef(P.S1, nullptr, wk.pc);
    rows_gemm<double, double, double>(P.W, P.ell, P.ell, P.ell, wk.pc, kp, wk.pl, P.S3, s);
    coef(P.S3, nullptr, wk.pc2);
    c = wk.pc2;
  } else {
    coef(P.S1, P.d, wk.pc);
  }
  rows_gemm<double, double, double>(P.V, A.n, P.ell, P.ldv, c, kp, wk.pq, P.S2, s);
}

template <class V>
static void blk_bwd(const BlkOp& A, const BlkPrec* P, int kp, double delta, BlkVecs<V> vec, GKState* st, BlkWork& wk,
                    hipStream_t s, bool pn_ready = false) {
  if (!pn_ready) blk_prod<V>(A, true, vec.u_top, kp, (V*)wk.pn, s);
  const unsigned g = blk_grid(A.n, kp);
  if (!P) {
    BLK_KP_SWITCH(kp, hipLaunchKernelGGL((k_blk_bwd<V, KP, true>), dim3(g), dim3(kBlock), 0, s, (const V*)wk.pn, A.Sn,
                                         A.n, delta, (const V*)vec.u_bot, vec.v, vec.g, (const GKState*)st,
                                         st + kp, (const double*)wk.beta_part, wk.beta_count, wk.alpha_part));
    wk.alpha_count = g;
    return;
  }
  BLK_KP_SWITCH(kp, hipLaunchKernelGGL((k_blk_bwd<V, KP, false>), dim3(g), dim3(kBlock), 0, s, (const V*)wk.pn, A.Sn,
                                       A.n, delta, (const V*)vec.u_bot, vec.v, vec.g, (const GKState*)st, st + kp,
                                       (const double*)wk.beta_part, wk.beta_count, wk.alpha_part));
  blk_pcoef<V>(A, *P, kp, vec.g, wk, s);
  BLK_KP_SWITCH(kp, hipLaunchKernelGGL((k_blk_pa_bwd<V, KP>), dim3(g), dim3(kBlock), 0, s, (const double*)wk.pq, P->S2,
                                       A.n, (const V*)vec.g, vec.v, (const GKState*)(st + kp), wk.alpha_part));
  wk.alpha_count = g;
}

template <class V>
void blk_phase_init(const BlkOp& Ares, const BlkOp& A, const BlkPrec* P, int kp, const double* B, const double* Bbot,
                    double bs, const double* X, bool x_zero, double delta, BlkVecs<V> vec, GKState* st, BlkWork& wk,
                    hipStream_t s, const double* r_ready) {
  APL_REQUIRE((!r_ready || std::is_same<V, double>::value), "blk_phase_init: a formed residual needs FP64 vectors");
  double* pm = (double*)wk.pm;
  const bool prod = !x_zero && !r_ready;
  if (prod) {
    if (Ares.f64)
      rows_gemm<double, double, double>((const double*)Ares.A, A.m, A.n, Ares.ld, X, kp, pm, Ares.Sm, s);
    else
      rows_gemm<float, double, double>((const float*)Ares.A, A.m, A.n, Ares.ld, X, kp, pm, Ares.Sm, s);
  }
  const unsigned g = blk_grid(std::max(A.m, A.n), kp);
  BLK_KP_SWITCH(kp, hipLaunchKernelGGL((k_blk_resid<V, KP>), dim3(g), dim3(kBlock), 0, s,
                                       (const double*)(prod ? pm : nullptr), Ares.Sm, A.m, A.n,
                                       r_ready ? r_ready : B, Bbot, bs, x_zero ? nullptr : X, delta, vec.u_top,
                                       vec.u_bot, wk.beta_part));
  wk.beta_count = g;
  fill_zero<V>(vec.y, A.n * kp, s);
  fill_zero<V>(vec.w, A.n * kp, s);
  blk_bwd<V>(A, P, kp, delta, vec, st, wk, s, r_ready != nullptr);
}

template <class V>
void blk_iteration(const BlkOp& A, const BlkPrec* P, int kp, double delta, BlkVecs<V> vec, GKState* st, BlkWork& wk,
                   hipStream_t s) {
  const unsigned g = blk_grid(std::max(A.m, A.n), kp);
  if (!P) {
    blk_prod<V>(A, false, vec.v, kp, (V*)wk.pm, s);
    BLK_KP_SWITCH(kp, hipLaunchKernelGGL((k_blk_fwd<V, KP, kFwdPlain>), dim3(g), dim3(kBlock), 0, s,
                                         (const V*)wk.pm, A.Sm, A.m, A.n, delta, (const V*)vec.v, vec.u_top,
                                         vec.u_bot, (const V*)vec.v, vec.w, vec.y, (const GKState*)(st + kp), st,
                                         (const double*)wk.alpha_part, wk.alpha_count, wk.beta_part));
  } else {
    blk_pcoef<V>(A, *P, kp, vec.v, wk, s);
    const unsigned gn = blk_grid(A.n, kp);
    BLK_KP_SWITCH(kp, hipLaunchKernelGGL((k_blk_pa_fwd<V, KP>), dim3(gn), dim3(kBlock), 0, s, (const double*)wk.pq,
                                         P->S2, A.n, (const V*)vec.v, vec.t, vec.w, vec.y, (const GKState*)(st + kp),
                                         st, (const double*)wk.alpha_part, wk.alpha_count));
    blk_prod<V>(A, false, vec.t, kp, (V*)wk.pm, s);
    BLK_KP_SWITCH(kp, hipLaunchKernelGGL((k_blk_fwd<V, KP, kFwdPre>), dim3(g), dim3(kBlock), 0, s, (const V*)wk.pm,
                                         A.Sm, A.m, A.n, delta, (const V*)vec.t, vec.u_top, vec.u_bot,
                                         (const V*)vec.v, vec.w, vec.y, (const GKState*)st, st,
                                         (const double*)nullptr, 0, wk.beta_part));
  }
  wk.beta_count = g;
  blk_bwd<V>(A, P, kp, delta, vec, st, wk, s);
}

template <class V>
void blk_phase_finish(const BlkOp& A, const BlkPrec* P, int kp, BlkVecs<V> vec, double* X, BlkWork& wk,
                      hipStream_t s) {
  const double* pq = nullptr;
  int S2 = 1;
  if (P) {
    blk_pcoef<V>(A, *P, kp, vec.y, wk, s);
    pq = wk.pq;
    S2 = P->S2;
  }
  hipLaunchKernelGGL((k_blk_add_x<V>), dim3(elem_grid(A.n * kp)), dim3(kBlock), 0, s, pq, S2, A.n * kp,
                     (const V*)vec.y, X);
}

int blk_norms(const BlkOp& A, int kp, int mode, const double* B, const double* Bbot, double bs, const double* X,
              double delta, double* tmp_m, double* tmp_n, BlkWork& wk, hipStream_t s, double* outv) {
  double* pn = (double*)wk.pn;
  if (mode == 0 || mode == 3) {
    const long long rows = mode == 0 ? A.m : A.n;
    const unsigned g = blk_grid(rows, kp);
    BLK_KP_SWITCH(kp, hipLaunchKernelGGL((k_blk_colsq<KP>), dim3(g), dim3(kBlock), 0, s, mode == 0 ? B : Bbot,
                                         (const double*)nullptr, 1, rows, 0.0, (const double*)nullptr, wk.norm_part,
                                         (double*)nullptr));
    return (int)g;
  }
  const double* top = B;
  const double* rbot = nullptr;
  if (mode == 2) {
    {
      double* pm = (double*)wk.pm;
      if (A.f64)
        rows_gemm<double, double, double>((const double*)A.A, A.m, A.n, A.ld, X, kp, pm, A.Sm, s);
      else
        rows_gemm<float, double, double>((const float*)A.A, A.m, A.n, A.ld, X, kp, pm, A.Sm, s);
      const unsigned g = blk_grid(std::max(A.m, A.n), kp);
      BLK_KP_SWITCH(kp, hipLaunchKernelGGL((k_blk_resid<double, KP>), dim3(g), dim3(kBlock), 0, s,
                                           (const double*)pm, A.Sm, A.m, A.n, B, Bbot, bs, X, delta, tmp_m, tmp_n,
                                           wk.beta_part));
      top = tmp_m;
      rbot = tmp_n;
    }
  }
  if (A.f64)
    rows_gemm<double, double, double>((const double*)A.At, A.n, A.m, A.ldt, top, kp, pn, A.Sn, s);
  else
    rows_gemm<float, double, double>((const float*)A.At, A.n, A.m, A.ldt, top, kp, pn, A.Sn, s);
  const unsigned g = blk_grid(A.n, kp);
  BLK_KP_SWITCH(kp, hipLaunchKernelGGL((k_blk_colsq<KP>), dim3(g), dim3(kBlock), 0, s, (const double*)nullptr,
                                       (const double*)pn, A.Sn, A.n, delta, rbot, wk.norm_part, outv));
  return (int)g;
}

template void blk_phase_init<double>(const BlkOp&, const BlkOp&, const BlkPrec*, int, const double*, const double*,
                                     double, const double*, bool, double, BlkVecs<double>, GKState*, BlkWork&,
                                     hipStream_t, const double*);
template void blk_phase_init<float>(const BlkOp&, const BlkOp&, const BlkPrec*, int, const double*, const double*,
                                    double, const double*, bool, double, BlkVecs<float>, GKState*, BlkWork&,
                                    hipStream_t, const double*);
template void blk_iteration<double>(const BlkOp&, const BlkPrec*, int, double, BlkVecs<double>, GKState*, BlkWork&,
                                    hipStream_t);
template void blk_iteration<float>(const BlkOp&, const BlkPrec*, int, double, BlkVecs<float>, GKState*, BlkWork&,
                                   hipStream_t);
template void blk_phase_finish<double>(const BlkOp&, const BlkPrec*, int, BlkVecs<double>, double*, BlkWork&,
                                       hipStream_t);
template void blk_phase_finish<float>(const BlkOp&, const BlkPrec*, int, BlkVecs<float>, double*, BlkWork&,
                                      hipStream_t);

}  // namespace aplicur
