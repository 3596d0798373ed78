// aplicur_sketch_noalloc: the sketch Y = S A of Alg. 3's initialisation
// (sparse sign embedding, Definition 5.1) into caller memory, for callers
// that cannot allocate device memory.  Same kernels as aplicur_sketch; its
// scratch is a fixed per-device array declared here.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "../../include/aplicur.h"
#include "kernels.h"

namespace aplicur {
void validate(const aplicur_mat* A, const aplicur_opts* o);
void set_last_error(const std::string& msg);

static size_t aligned256(size_t bytes) { return (std::max<size_t>(bytes, 1) + 255) / 256 * 256; }

template <class F>
static int guarded_na(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return APLICUR_E_HIP;
  } catch (...) {
    set_last_error("unknown error");
    return APLICUR_E_HIP;
  }
}

// ------------------------------------------------------------------ sketch without allocation
// Device memory of aplicur_sketch_noalloc: one fixed array per device (each
// device that runs the library holds its own copy until the process ends).
// Host code takes its address once per device with hipGetSymbolAddress and
// only ever passes that address to kernels: the symbol itself names a host
// stand-in, not device memory.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
static std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
static void* g_scratch_dev[kMaxDevices] = {};

static char* scratch_of_current_device() {
  int dev = 0;
  APL_HIP(hipGetDevice(&dev));
  APL_REQUIRE(dev >= 0 && dev < kMaxDevices, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    APL_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    APL_REQUIRE(p != nullptr, "no device address for the scratch array");
    g_scratch_dev[dev] = p;
  }
  return (char*)g_scratch_dev[dev];
}

// Scratch layout of one call: sketch rows and signs, then (CSR) the
// validation flag and the CSR of A^T, or (dense) the inverse of the
// embedding (per target row, the rows of A it sums).
struct NoAllocPlan {
  int s = 0, xi = 0;
  size_t rows = 0, neg = 0, bad = 0, tp = 0, ti = 0, tv = 0, tsc = 0, part = 0, total = 0;
};

static NoAllocPlan plan_noalloc(const aplicur_mat* A, const aplicur_opts* o) {
  NoAllocPlan p;
  const long long m = A->m, n = A->n;
  int s_rows = (int)std::ceil(1.1 * o->block - 1e-12);
  p.s = (int)std::max<long long>(1, std::min<long long>(s_rows, m));
  p.xi = std::min(o->xi > 0 ? o->xi : 8, p.s);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += aligned256(bytes);
    return at;
  };
  p.rows = take(sizeof(uint16_t) * (size_t)m * p.xi);
  p.neg = take((size_t)m);
  const size_t vs = A->dtype == APLICUR_F64 ? 8 : 4;
  if (A->format == APLICUR_CSR) {
    p.bad = take(sizeof(int));
    p.tp = take(sizeof(int) * (size_t)(n + 1));
    p.ti = take(sizeof(int) * (size_t)std::max<long long>(1, A->nnz));
    p.tv = take(vs * (size_t)std::max<long long>(1, A->nnz));
    p.tsc = take(sizeof(int) * (size_t)n);
  } else {
    p.part = take(sketch_dense_scratch(m, p.s, p.xi));
  }
  p.total = off;
  return p;
}
}  // namespace aplicur

using namespace aplicur;

extern "C" {

int aplicur_sketch_noalloc(const aplicur_mat* A, const aplicur_opts* opts, double* Y, void* stream) {
  return guarded_na([&]() {
    validate(A, opts);
    APL_REQUIRE(Y, "Y is null");
    APL_REQUIRE(opts->precond != 0, "the sketch belongs to APLICUR: precond must be 1 or 2");
    APL_REQUIRE(opts->sketch == 0, "only the sparse sign sketch (sketch = 0) runs without allocation");
    APL_REQUIRE(A->format != APLICUR_DENSE_COL,
                "column-major A needs a row-major copy: pass it row-major (APLICUR_DENSE) or as CSR");
    const NoAllocPlan p = plan_noalloc(A, opts);
    APL_REQUIRE(p.total <= kNoAllocScratchBytes,
                "this sketch needs " + std::to_string(p.total) + " bytes of scratch; aplicur_sketch_noalloc has " +
                    std::to_string(kNoAllocScratchBytes) + " (use aplicur_sketch)");
    hipStream_t s = (hipStream_t)stream;
    char* base = scratch_of_current_device();
    uint16_t* rows = (uint16_t*)(base + p.rows);
    uint8_t* neg = (uint8_t*)(base + p.neg);
    const long long m = A->m, n = A->n;
    const bool f64 = A->dtype == APLICUR_F64;
    if (A->format == APLICUR_CSR) {
      int* tp = (int*)(base + p.tp);
      int* ti = (int*)(base + p.ti);
      void* tv = base + p.tv;
      int* tsc = (int*)(base + p.tsc);
      const int code = check_csr(A->row_ptr, A->col_idx, m, n, A->nnz, (int*)(base + p.bad), s);
      APL_REQUIRE(code == 0, code & 1 ? "CSR row_ptr is malformed" : "CSR col_idx out of range");
      if (f64)
        launch_csr_transpose<double>(A->row_ptr, A->col_idx, (const double*)A->val, m, n, A->nnz, tp, ti,
                                     (double*)tv, tsc, s);
      else
        launch_csr_transpose<float>(A->row_ptr, A->col_idx, (const float*)A->val, m, n, A->nnz, tp, ti,
                                    (float*)tv, tsc, s);
      launch_gen_sketch(opts->seed, p.s, m, p.xi, rows, neg, s);
      if (f64)
        launch_sketch_csr<double>(tp, ti, (const double*)tv, n, p.s, p.xi, rows, neg, Y, s);
      else
        launch_sketch_csr<float>(tp, ti, (const float*)tv, n, p.s, p.xi, rows, neg, Y, s);
    } else {
      void* part = base + p.part;
      launch_gen_sketch(opts->seed, p.s, m, p.xi, rows, neg, s);
      if (f64)
        launch_sketch_dense<double>((const double*)A->val, m, n, A->ld, p.s, p.xi, rows, neg, Y, part, s);
      else
        launch_sketch_dense<float>((const float*)A->val, m, n, A->ld, p.s, p.xi, rows, neg, Y, part, s);
    }
    APL_HIP(hipGetLastError());
    return APLICUR_OK;
  });
}

}  // extern "C"
