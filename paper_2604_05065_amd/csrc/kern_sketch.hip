// One-time set-up kernels: the method's random stream (sparse sign embedding,
// Definition 5.1; Gaussian probes of the 2-norm bound, Sec. 5.3.1), the CSR
// transpose used for coalesced A^T products, and the sketch Y = S A (Alg. 3,
// initialisation), computed once and reused for every rank increment.
#include "kernels.h"

namespace aplicur {

// SplitMix64 (Steele, Lea, Flood 2014), variant-13 finalizer.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
__device__ __forceinline__ uint64_t stream_key(uint64_t seed, uint64_t stream) {
  return mix64(seed + kGolden * (stream + 1));
}
__device__ __forceinline__ uint64_t draw(uint64_t key, uint64_t ctr) {
  return mix64(key + kGolden * (ctr + 1));
}

// Column i of S (the coefficients applied to row i of A): xi distinct rows of
// [0, s) by redraw-on-repeat (64 attempts, then the smallest unused row) and a
// Rademacher sign each (top bit of a stream-1 draw).
__global__ void k_gen_sketch(uint64_t seed, int s, long long m, int xi, uint16_t* rows,
                             uint8_t* negmask) {
  long long i = blockIdx.x * (long long)kBlock + threadIdx.x;
  if (i >= m) return;
  const uint64_t k0 = stream_key(seed, 0), k1 = stream_key(seed, 1);
  int chosen[8];
  unsigned neg = 0;
  for (int t = 0; t < xi; ++t) {
    int h = -1;
    for (int a = 0; a < 64 && h < 0; ++a) {
      int cand = (int)(draw(k0, ((uint64_t)i * 8 + t) * 64 + a) % (uint64_t)s);
      bool clash = false;
      for (int tp = 0; tp < t; ++tp) clash |= (chosen[tp] == cand);
      if (!clash) h = cand;
    }
    if (h < 0) {
      for (int r = 0; r < s && h < 0; ++r) {
        bool used = false;
        for (int tp = 0; tp < t; ++tp) used |= (chosen[tp] == r);
        if (!used) h = r;
      }
    }
    chosen[t] = h;
    rows[i * xi + t] = (uint16_t)h;
    if (draw(k1, (uint64_t)i * 8 + t) >> 63) neg |= 1u << t;
  }
  negmask[i] = (uint8_t)neg;
}

// Probe vectors W (n x r, column-major): Box-Muller on two 53-bit uniforms.
__global__ void k_gen_probes(uint64_t seed, long long n, int r, double* W) {
  long long idx = blockIdx.x * (long long)kBlock + threadIdx.x;
  if (idx >= n * r) return;
  const uint64_t k2 = stream_key(seed, 2);
  const uint64_t c = (uint64_t)idx;  // = i * n + j for column i, component j
  uint64_t d0 = draw(k2, 2 * c), d1 = draw(k2, 2 * c + 1);
  double u1 = ((double)(d0 >> 11) + 1.0) * 0x1.0p-53;
  double u2 = (double)(d1 >> 11) * 0x1.0p-53;
  W[idx] = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

// Gaussian sketch S (s x m, column-major): entry (h, i) the Box-Muller normal
// of the stream-3 draws 2c and 2c + 1, c = i s + h, divided by sqrt(s).
__global__ void k_gen_gauss_sketch(uint64_t seed, int s, long long m, double* S) {
  const long long idx = blockIdx.x * (long long)kBlock + threadIdx.x;
  if (idx >= m * s) return;
  const uint64_t k3 = stream_key(seed, 3);
  const uint64_t c = (uint64_t)idx;
  const uint64_t d0 = draw(k3, 2 * c), d1 = draw(k3, 2 * c + 1);
  const double u1 = ((double)(d0 >> 11) + 1.0) * 0x1.0p-53;
  const double u2 = (double)(d1 >> 11) * 0x1.0p-53;
  S[idx] = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2) / sqrt((double)s);
}

void launch_gen_gauss_sketch(uint64_t seed, int s, long long m, double* S, hipStream_t st) {
  hipLaunchKernelGGL(k_gen_gauss_sketch, dim3(ceil_div(m * s, kBlock)), dim3(kBlock), 0, st, seed, s, m, S);
}

// Y(:, j) = S A(:, j) for CSR A through the CSR of A^T (row j lists the
// entries of column j of A in row order): one wave per j, lane h < s sums
// a_ij S(h, i) over the column's entries in order; Y row-major s x n.
template <class T>
__global__ void __launch_bounds__(kBlock)
    k_sketch_gauss_csr(const int* __restrict__ t_ptr, const int* __restrict__ t_idx, const T* __restrict__ t_val,
                       long long n, int s, const double* __restrict__ S, double* __restrict__ Y) {
  const long long j = blockIdx.x * (long long)(kBlock / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (j >= n) return;
  const int e0 = t_ptr[j], e1 = t_ptr[j + 1];
  for (int h0 = 0; h0 < s; h0 += kWave) {
    const int h = h0 + lane;
    double acc = 0.0;
    if (h < s)
      for (int e = e0; e < e1; ++e) acc += (double)t_val[e] * S[(long long)t_idx[e] * s + h];
    if (h < s) Y[(long long)h * n + j] = acc;
  }
}

template <class T>
void launch_sketch_gauss_csr(const int* t_ptr, const int* t_idx, const T* t_val, long long n, int s, const double* S,
                             double* Y, hipStream_t st) {
  hipLaunchKernelGGL((k_sketch_gauss_csr<T>), dim3(ceil_div(n, kBlock / kWave)), dim3(kBlock), 0, st, t_ptr, t_idx,
                     t_val, n, s, S, Y);
}
template void launch_sketch_gauss_csr<double>(const int*, const int*, const double*, long long, int, const double*,
                                              double*, hipStream_t);
template void launch_sketch_gauss_csr<float>(const int*, const int*, const float*, long long, int, const double*,
                                             double*, hipStream_t);

__global__ void k_widen(const float* __restrict__ a, double* __restrict__ b, long long count) {
  for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < count; i += (long long)gridDim.x * kBlock)
    b[i] = (double)a[i];
}

void widen(const float* a, double* b, long long count, hipStream_t st) {
  hipLaunchKernelGGL(k_widen, dim3((unsigned)std::min<long long>(ceil_div(count, kBlock), 4096)), dim3(kBlock), 0,
                     st, a, b, count);
}

void launch_gen_sketch(uint64_t seed, int s, long long m, int xi, uint16_t* rows,
                       uint8_t* negmask, hipStream_t st) {
  hipLaunchKernelGGL(k_gen_sketch, dim3(ceil_div(m, kBlock)), dim3(kBlock), 0, st, seed, s, m,
                     xi, rows, negmask);
}

void launch_gen_probes(uint64_t seed, long long n, int r, double* W, hipStream_t st) {
  hipLaunchKernelGGL(k_gen_probes, dim3(ceil_div(n * r, kBlock)), dim3(kBlock), 0, st, seed,
                     n, r, W);
}

// ---------------------------------------------------------------- CSR validation
// bad[0] |= 1 for a malformed row pointer, 2 for a column index out of range.
__global__ void k_check_csr(const int* row_ptr, const int* col_idx, long long m, long long n, long long nnz,
                            int* bad) {
  long long i = blockIdx.x * (long long)kBlock + threadIdx.x;
  if (i >= m) return;
  const long long b = row_ptr[i], e = row_ptr[i + 1];
  if ((i == 0 && b != 0) || b < 0 || e < b || e > nnz || (i == m - 1 && e != nnz)) {
    atomicOr(bad, 1);
    return;
  }
  for (long long k = b; k < e; ++k) {
    const int c = col_idx[k];
    if (c < 0 || c >= n) {
      atomicOr(bad, 2);
      return;
    }
  }
}

// p[0..count) = 0 (a kernel, not a memset, so that a captured graph may hold it).
__global__ void k_zero_int(int* p, long long count) {
  for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < count; i += (long long)gridDim.x * kBlock)
    p[i] = 0;
}

static void zero_int(int* p, long long count, hipStream_t st) {
  if (count <= 0) return;
  const long long g = (count + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_zero_int, dim3((unsigned)(g < 1024 ? g : 1024)), dim3(kBlock), 0, st, p, count);
}

int check_csr(const int* row_ptr, const int* col_idx, long long m, long long n, long long nnz, int* bad_dev,
              hipStream_t st) {
  zero_int(bad_dev, 1, st);
  hipLaunchKernelGGL(k_check_csr, dim3(ceil_div(m, kBlock)), dim3(kBlock), 0, st, row_ptr, col_idx, m, n, nnz,
                     bad_dev);
  int h = 0;
  APL_HIP(hipMemcpyAsync(&h, bad_dev, sizeof(int), hipMemcpyDeviceToHost, st));
  APL_HIP(hipStreamSynchronize(st));
  return h;
}

// ---------------------------------------------------------------- CSR transpose
__global__ void k_count_cols(const int* col_idx, long long nnz, int* counts) {
  long long k = blockIdx.x * (long long)kBlock + threadIdx.x;
  if (k < nnz) atomicAdd(&counts[col_idx[k]], 1);
}

// Exclusive scan of counts[0..n) into ptr[0..n], one workgroup, sequential
// chunks with a block-wide scan inside each chunk.
__global__ void k_scan_single(const int* counts, int n, int* ptr) {
  __shared__ int buf[kBlock];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < n; base += kBlock) {
    int i = base + threadIdx.x;
    int v = (i < n) ? counts[i] : 0;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
      int add = (threadIdx.x >= off) ? buf[threadIdx.x - off] : 0;
      __syncthreads();
      buf[threadIdx.x] += add;
      __syncthreads();
    }
    if (i < n) ptr[i] = carry + buf[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == kBlock - 1) carry += buf[kBlock - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) ptr[n] = carry;
}

template <class T>
__global__ void k_fill_transpose(const int* row_ptr, const int* col_idx, const T* val, long long m,
                                 int* cursor, int* t_idx, T* t_val) {
  long long i = blockIdx.x * (long long)kBlock + threadIdx.x;
  if (i >= m) return;
  for (int k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
    int c = col_idx[k];
    int pos = atomicAdd(&cursor[c], 1);
    t_idx[pos] = (int)i;
    t_val[pos] = val[k];
  }
}

// Sort each row of the transpose by column (original row) index so that the
// summation order of every A^T product is fixed.
template <class T>
__global__ void k_sort_segments(const int* ptr, long long n, int* idx, T* val) {
  long long j = blockIdx.x * (long long)kBlock + threadIdx.x;
  if (j >= n) return;
  int b = ptr[j], e = ptr[j + 1];
  for (int a = b + 1; a < e; ++a) {
    int key = idx[a];
    T v = val[a];
    int p = a - 1;
    while (p >= b && idx[p] > key) {
      idx[p + 1] = idx[p];
      val[p + 1] = val[p];
      --p;
    }
    idx[p + 1] = key;
    val[p + 1] = v;
  }
}

template <class T>
void launch_csr_transpose(const int* row_ptr, const int* col_idx, const T* val, long long m,
                          long long n, long long nnz, int* t_ptr, int* t_idx, T* t_val,
                          int* scratch_n, hipStream_t st) {
  zero_int(scratch_n, n, st);
  if (nnz > 0)
    hipLaunchKernelGGL(k_count_cols, dim3(ceil_div(nnz, kBlock)), dim3(kBlock), 0, st, col_idx,
                       nnz, scratch_n);
  hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(kBlock), 0, st, scratch_n, (int)n, t_ptr);
  APL_HIP(hipMemcpyAsync(scratch_n, t_ptr, sizeof(int) * n, hipMemcpyDeviceToDevice, st));
  if (m > 0)
    hipLaunchKernelGGL(k_fill_transpose<T>, dim3(ceil_div(m, kBlock)), dim3(kBlock), 0, st, row_ptr,
                       col_idx, val, m, scratch_n, t_idx, t_val);
  if (n > 0)
    hipLaunchKernelGGL(k_sort_segments<T>, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, st, t_ptr, n,
                       t_idx, t_val);
}
template void launch_csr_transpose<float>(const int*, const int*, const float*, long long,
                                          long long, long long, int*, int*, float*, int*,
                                          hipStream_t);
template void launch_csr_transpose<double>(const int*, const int*, const double*, long long,
                                           long long, long long, int*, int*, double*, int*,
                                           hipStream_t);

// ---------------------------------------------------------------- row subset of a CSR matrix
__global__ void k_rows_len(const int* rp, const int* I, int ell, int* len) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k < ell) len[k] = rp[I[k] + 1] - rp[I[k]];
}

template <class T>
__global__ void k_copy_rows(const int* rp, const int* ci, const T* val, const int* I, int ell, const int* r_ptr,
                            int* r_idx, double* r_val) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= ell) return;
  const int src = rp[I[k]], len = rp[I[k] + 1] - src, dst = r_ptr[k];
  for (int e = 0; e < len; ++e) {
    r_idx[dst + e] = ci[src + e];
    r_val[dst + e] = (double)val[src + e];
  }
}

template <class T>
long long launch_gather_csr_rows(const int* row_ptr, const int* col_idx, const T* val, const int* I, int ell,
                                 int* r_ptr, int* r_idx, double* r_val, long long cap, int* scratch,
                                 hipStream_t st) {
  const unsigned g = ceil_div(ell > 0 ? ell : 1, kBlock);
  if (ell > 0) hipLaunchKernelGGL(k_rows_len, dim3(g), dim3(kBlock), 0, st, row_ptr, I, ell, scratch);
  hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(kBlock), 0, st, (const int*)scratch, ell, r_ptr);
  int nnz = 0;
  APL_HIP(hipMemcpyAsync(&nnz, r_ptr + ell, sizeof(int), hipMemcpyDeviceToHost, st));
  APL_HIP(hipStreamSynchronize(st));
  if (nnz > cap) throw Error(-1, "row subset exceeds its reserved capacity");
  if (ell > 0)
    hipLaunchKernelGGL(k_copy_rows<T>, dim3(g), dim3(kBlock), 0, st, row_ptr, col_idx, val, I, ell,
                       (const int*)r_ptr, r_idx, r_val);
  return nnz;
}
template long long launch_gather_csr_rows<float>(const int*, const int*, const float*, const int*, int, int*, int*,
                                                 double*, long long, int*, hipStream_t);
template long long launch_gather_csr_rows<double>(const int*, const int*, const double*, const int*, int, int*,
                                                  int*, double*, long long, int*, hipStream_t);

// ---------------------------------------------------------------- sketch, CSR A
// Y(:, j) = sum over the non-zeros (i, a) of column j of A of S(:, i) a.
// One wave per 64 columns; lane l owns column j0 + l and accumulates it in a
// private LDS column of s doubles, walking the sorted transpose row in order,
// so the sum order is fixed.
template <class T>
__global__ void __launch_bounds__(kWave) k_sketch_csr(const int* t_ptr, const int* t_idx,
                                                      const T* t_val, long long n, int s, int xi,
                                                      const uint16_t* rows, const uint8_t* negmask,
                                                      double scale, double* Y) {
#pragma clang fp contract(off)
  extern __shared__ double lds[];  // s x 64
  const int l = threadIdx.x;
  const long long j = blockIdx.x * (long long)kWave + l;
  for (int h = 0; h < s; ++h) lds[h * kWave + l] = 0.0;
  if (j < n) {
    for (int k = t_ptr[j]; k < t_ptr[j + 1]; ++k) {
      const long long i = t_idx[k];
      const double a = (double)t_val[k] * scale;
      const unsigned neg = negmask[i];
      for (int t = 0; t < xi; ++t) {
        const int h = rows[i * xi + t];
        lds[h * kWave + l] += ((neg >> t) & 1u) ? -a : a;
      }
    }
    for (int h = 0; h < s; ++h) Y[(long long)h * n + j] = lds[h * kWave + l];
  }
}

template <class T>
void launch_sketch_csr(const int* t_ptr, const int* t_idx, const T* t_val, long long n, int s,
                       int xi, const uint16_t* rows, const uint8_t* negmask, double* Y,
                       hipStream_t st) {
  size_t lds = sizeof(double) * s * kWave;
  APL_REQUIRE(lds <= 160 * 1024, "sketch dimension too large for the LDS strip");
  APL_HIP(hipFuncSetAttribute((const void*)k_sketch_csr<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(k_sketch_csr<T>, dim3(ceil_div(n, kWave)), dim3(kWave), lds, st, t_ptr, t_idx,
                     t_val, n, s, xi, rows, negmask, 1.0 / sqrt((double)xi), Y);
}
template void launch_sketch_csr<float>(const int*, const int*, const float*, long long, int, int,
                                       const uint16_t*, const uint8_t*, double*, hipStream_t);
template void launch_sketch_csr<double>(const int*, const int*, const double*, long long, int, int,
                                        const uint16_t*, const uint8_t*, double*, hipStream_t);

// ---------------------------------------------------------------- sketch, dense A
// Y(h, :) = sum over the rows i of A that S sends to target row h of
// +-scale A(i, :), the rows taken in increasing i: each entry is the same
// row-order sum of the same rounded terms as in the CSR sketch.  Three small
// kernels first build the inverse of the embedding (for every target row h,
// the list of (i, sign) in increasing i, as a counting sort over 256-row
// chunks of A), then one wave per (h, 256-column strip) accumulates its
// strip in FP64 registers, reading the rows of its list.  Each row of A is
// read by the xi waves of its targets; the workgroups of one strip go to one
// XCD (workgroup ids reach the XCDs round robin), whose waves walk their lists
// in step, so the rows they share are read from HBM once and from L2 after.
constexpr int kInvRows = 256;          // rows of A per chunk of the inverse map
constexpr int kSgW = 4;                // waves per gather workgroup (one target row each)
constexpr int kSgCols = 4 * kWave;     // columns per strip (four per lane)
constexpr int kSgU = 8;                // rows in flight per wave
constexpr int kXcds = 8;

struct SketchInv {
  int* cnt;   // nchunk x s: per-chunk counts, then their exclusive prefix over chunks
  int* tot;   // s: list lengths
  int* ptr;   // s + 1: list offsets
  int* list;  // m xi: 2 i + (1 if the sign is negative), grouped by target row
};

static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

static SketchInv carve_inv(void* scratch, long long m, int s, int xi) {
  const long long nchunk = (m + kInvRows - 1) / kInvRows;
  char* p = (char*)scratch;
  SketchInv v;
  v.cnt = (int*)p;
  p += al256(sizeof(int) * (size_t)nchunk * s);
  v.tot = (int*)p;
  p += al256(sizeof(int) * (size_t)s);
  v.ptr = (int*)p;
  p += al256(sizeof(int) * (size_t)(s + 1));
  v.list = (int*)p;
  return v;
}

size_t sketch_dense_scratch(long long m, int s, int xi) {
  const long long nchunk = (m + kInvRows - 1) / kInvRows;
  return al256(sizeof(int) * (size_t)nchunk * s) + al256(sizeof(int) * (size_t)s) +
         al256(sizeof(int) * (size_t)(s + 1)) + al256(sizeof(int) * (size_t)m * xi);
}

// count of target h among the chunk's rows, for every h < s
__global__ void __launch_bounds__(kBlock) k_inv_count(const uint16_t* rows, long long m, int s, int xi, int* cnt) {
  __shared__ uint16_t tg[kInvRows * 8];
  const long long i0 = blockIdx.x * (long long)kInvRows;
  const int ne = (int)min((long long)kInvRows, m - i0) * xi;
  for (int e = threadIdx.x; e < ne; e += kBlock) tg[e] = rows[i0 * xi + e];
  __syncthreads();
  for (int h = threadIdx.x; h < s; h += kBlock) {
    int c = 0;
    for (int e = 0; e < ne; ++e) c += tg[e] == h;
    cnt[blockIdx.x * (long long)s + h] = c;
  }
}

// per target row: exclusive prefix of its counts over the chunks, and the total
__global__ void k_inv_prefix(int* cnt, long long nchunk, int s, int* tot) {
  const int h = blockIdx.x * kBlock + threadIdx.x;
  if (h >= s) return;
  int acc = 0;
  for (long long c = 0; c < nchunk; ++c) {
    const int v = cnt[c * s + h];
    cnt[c * s + h] = acc;
    acc += v;
  }
  tot[h] = acc;
}

// each target row's entries of the chunk, in row order, at its place in the list
__global__ void __launch_bounds__(kBlock) k_inv_fill(const uint16_t* rows, const uint8_t* negmask, long long m,
                                                     int s, int xi, const int* cnt, const int* ptr, int* list) {
  __shared__ uint16_t tg[kInvRows * 8];
  __shared__ uint8_t ng[kInvRows];
  const long long i0 = blockIdx.x * (long long)kInvRows;
  const int nr = (int)min((long long)kInvRows, m - i0), ne = nr * xi;
  for (int e = threadIdx.x; e < ne; e += kBlock) tg[e] = rows[i0 * xi + e];
  for (int r = threadIdx.x; r < nr; r += kBlock) ng[r] = negmask[i0 + r];
  __syncthreads();
  for (int h = threadIdx.x; h < s; h += kBlock) {
    int pos = ptr[h] + cnt[blockIdx.x * (long long)s + h];
    for (int e = 0; e < ne; ++e) {
      if (tg[e] == h) {
        const int r = e / xi, t = e - r * xi;
        list[pos++] = (int)(2 * (i0 + r)) + ((ng[r] >> t) & 1);
      }
    }
  }
}

template <class T>
struct Quad;
template <>
struct Quad<float> {
  float v[4];
};
template <>
struct Quad<double> {
  double v[4];
};

// four consecutive elements of a row; VEC: the address is 16-byte aligned
// (FP32) or the two halves are (FP64), and all four lie inside the row
template <class T, bool VEC>
__device__ __forceinline__ Quad<T> load_quad(const T* p, long long j, long long n) {
  Quad<T> q;
  if constexpr (VEC) {
    if constexpr (sizeof(T) == 4) {
      const float4 f = *(const float4*)(p + j);
      q.v[0] = f.x; q.v[1] = f.y; q.v[2] = f.z; q.v[3] = f.w;
    } else {
      const double2 f0 = *(const double2*)(p + j), f1 = *(const double2*)(p + j + 2);
      q.v[0] = f0.x; q.v[1] = f0.y; q.v[2] = f1.x; q.v[3] = f1.y;
    }
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) q.v[c] = p[min(j + c, n - 1)];
  }
  return q;
}

// kSgU rows of a list (the first cnt of them when TAIL), their loads issued
// before the first add; the adds go in list order
template <class T, bool VEC, bool TAIL>
__device__ __forceinline__ void gather_batch(const T* A, long long ld, long long n, long long jl, const int* lp,
                                             int cnt, double scale, double (&acc)[4]) {
#pragma clang fp contract(off)
  int code[kSgU];
#pragma unroll
  for (int u = 0; u < kSgU; ++u) code[u] = lp[TAIL ? min(u, cnt - 1) : u];
  Quad<T> a[kSgU];
#pragma unroll
  for (int u = 0; u < kSgU; ++u) a[u] = load_quad<T, VEC>(A + (long long)(code[u] >> 1) * ld, jl, n);
#pragma unroll
  for (int u = 0; u < kSgU; ++u) {
    if (!TAIL || u < cnt) {
      const double sc = (code[u] & 1) ? -scale : scale;
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] += (double)a[u].v[c] * sc;
    }
  }
}

template <class T, bool VEC>
__global__ void __launch_bounds__(kSgW * kWave) k_sketch_gather(const T* A, long long n, long long ld, int s,
                                                                const int* ptr, const int* list, double scale,
                                                                int strips, int hgroups, double* Y) {
#pragma clang fp contract(off)
  const int k = blockIdx.x / kXcds;
  const int strip = (k / hgroups) * kXcds + (int)(blockIdx.x % kXcds);
  const int h = (k % hgroups) * kSgW + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  if (strip >= strips || h >= s) return;
  const int lane = threadIdx.x % kWave;
  const long long j = (long long)strip * kSgCols + 4 * lane;
  const long long jl = j < n ? j : 0;  // lanes past the end read a valid quad and store nothing
  const int p0 = ptr[h], p1 = ptr[h + 1];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int p = p0;
  for (; p + kSgU <= p1; p += kSgU) gather_batch<T, VEC, false>(A, ld, n, jl, list + p, kSgU, scale, acc);
  if (p < p1) gather_batch<T, VEC, true>(A, ld, n, jl, list + p, p1 - p, scale, acc);
  double* y = Y + (long long)h * n;
#pragma unroll
  for (int c = 0; c < 4; ++c)
    if (j + c < n) y[j + c] = acc[c];
}

template <class T>
void launch_sketch_dense(const T* A, long long m, long long n, long long ld, int s, int xi, const uint16_t* rows,
                         const uint8_t* negmask, double* Y, void* scratch, hipStream_t st) {
  APL_REQUIRE(m < (1LL << 30), "the dense sparse-sign sketch takes fewer than 2^30 rows");
  APL_REQUIRE(xi >= 1 && xi <= 8, "xi must be in [1, 8]");
  const long long nchunk = (m + kInvRows - 1) / kInvRows;
  const SketchInv v = carve_inv(scratch, m, s, xi);
  hipLaunchKernelGGL(k_inv_count, dim3((unsigned)nchunk), dim3(kBlock), 0, st, rows, m, s, xi, v.cnt);
  hipLaunchKernelGGL(k_inv_prefix, dim3(ceil_div(s, kBlock)), dim3(kBlock), 0, st, v.cnt, nchunk, s, v.tot);
  hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(kBlock), 0, st, (const int*)v.tot, s, v.ptr);
  hipLaunchKernelGGL(k_inv_fill, dim3((unsigned)nchunk), dim3(kBlock), 0, st, rows, negmask, m, s, xi,
                     (const int*)v.cnt, (const int*)v.ptr, v.list);
  if (n == 0) return;
  const int strips = (int)ceil_div(n, kSgCols), hgroups = (int)ceil_div(s, kSgW);
  const long long grid = (long long)ceil_div(strips, kXcds) * kXcds * hgroups;
  APL_REQUIRE(grid < (1LL << 31), "sketch grid too large");
  const double scale = 1.0 / sqrt((double)xi);
  const bool vec = (ld % 4 == 0) && (n % 4 == 0) && ((uintptr_t)A % 16 == 0);
  if (vec)
    hipLaunchKernelGGL((k_sketch_gather<T, true>), dim3((unsigned)grid), dim3(kSgW * kWave), 0, st, A, n, ld, s,
                       (const int*)v.ptr, (const int*)v.list, scale, strips, hgroups, Y);
  else
    hipLaunchKernelGGL((k_sketch_gather<T, false>), dim3((unsigned)grid), dim3(kSgW * kWave), 0, st, A, n, ld, s,
                       (const int*)v.ptr, (const int*)v.list, scale, strips, hgroups, Y);
}
template void launch_sketch_dense<float>(const float*, long long, long long, long long, int, int, const uint16_t*,
                                         const uint8_t*, double*, void*, hipStream_t);
template void launch_sketch_dense<double>(const double*, long long, long long, long long, int, int,
                                          const uint16_t*, const uint8_t*, double*, void*, hipStream_t);

}  // namespace aplicur
