// Shared definitions of the APLICUR HIP library (gfx950 / CDNA4, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>

namespace aplicur {

constexpr int kBlock = 256;  // threads per workgroup everywhere (4 wave64s)
constexpr int kWave = 64;

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define APL_HIP(x)                                                                     \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess)                                                              \
      throw ::aplicur::Error(-3, std::string(#x) + ": " + hipGetErrorString(e_) + " (" + \
                                     __FILE__ + ":" + std::to_string(__LINE__) + ")"); \
  } while (0)

#define APL_REQUIRE(cond, msg)                                   \
  do {                                                           \
    if (!(cond)) throw ::aplicur::Error(-1, std::string(msg));   \
  } while (0)

// Stop reasons of an LSQR phase (same numbering as the oracle).
enum StopReason { kStopNone = 0, kStopMetric = 1, kStopLsqr = 2, kStopDynamic = 3,
                  kStopBudget = 4, kStopExact = 5 };

// Per right-hand-side state of one Golub-Kahan / LSQR phase, FP64 in every
// precision mode.  Lives in device memory as two slots (see kern_gk.hip):
// the kernel that finishes alpha writes slot 0, the one that finishes beta
// writes slot 1.  Vectors are kept unnormalised: u = u_raw / beta,
// v = v_raw / alpha, and the y/w update of iteration j is applied lazily by
// the first kernel of iteration j + 1.
struct GKState {
  double alpha, beta;          // norms of the current raw v and u
  double rhobar, phibar;       // Givens QR state
  double anorm2;               // running ||A~||_F^2 estimate
  double phibar_prev, rate1;   // dynamic stopping history
  double coef_y, coef_w;       // pending y += coef_y w ; w = v - coef_w w
  double arnorm;               // ||A~^T r|| estimate
  double pnorm;                // ||P|| (1 without a preconditioner)
  double tol_abs;              // tol_ne * ||A^T b||
  double eps_lsqr, baug_eps;   // Paige-Saunders tolerance and eps * ||b_aug||
  double nu, sigma_l;          // dynamic rule (nu = +inf disables it)
  double delta;                // sqrt(mu)
  double h2;                   // ||A_mu^T r||^2 at phase start (normal-equation residual)
  double beta1;                // initial residual of the phase
  double rel_tol;              // phase ends when ||A~^T r|| <= rel_tol * its start (low-precision phases; 0: off)
  int iter, max_iter, stop, reason, pending, have_rate1, init, pad;
};

// ---------------------------------------------------------------- device helpers
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// v from lane src of the wave (src uniform)
__device__ __forceinline__ double lane_bcast(double v, int src) {
  const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)bits, src);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(bits >> 32), src);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the whole workgroup (kBlock threads); result valid in thread 0.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[kBlock / kWave];
  v = wave_sum(v);
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < kBlock / kWave; ++i) s += red[i];
  }
  return s;
}

inline unsigned ceil_div(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

}  // namespace aplicur
