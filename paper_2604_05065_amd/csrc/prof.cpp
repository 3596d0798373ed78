// Event timing of the blocked product kernel inside solves, for measurement:
// while switched on, every dispatch of the row-streaming product kernel of
// the several-right-hand-side path (dense A) carries a HIP event pair that
// takes the kernel's own start and end, so a caller can read the mean
// duration of the launches a solve made without a profiler.  The events are
// created on first use and reused afterwards (a warm-up with timing on makes
// them before a timed region); reading them waits for the recorded launches.
#include <mutex>
#include <string>
#include <vector>

#include "../../include/aplicur.h"
#include "prof.h"

namespace aplicur {
void set_last_error(const std::string& msg);

namespace {
struct ProdProf {
  std::mutex mu;
  bool on = false;
  int device = -1;
  std::vector<hipEvent_t> pool;  // 2 per launch, kept for reuse
  std::vector<int> kind;         // kind of each recorded launch
  long long untimed[kProfKinds] = {};
};
ProdProf g_prof;
constexpr size_t kProfMaxLaunches = 65536;
}  // namespace

bool prof_take(int kind, hipEvent_t* e0, hipEvent_t* e1) {
  std::lock_guard<std::mutex> g(g_prof.mu);
  if (!g_prof.on || kind < 0 || kind >= kProfKinds) return false;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != g_prof.device || g_prof.kind.size() >= kProfMaxLaunches) {
    ++g_prof.untimed[kind];
    return false;
  }
  const size_t at = 2 * g_prof.kind.size();
  while (g_prof.pool.size() < at + 2) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) {
      ++g_prof.untimed[kind];
      return false;
    }
    g_prof.pool.push_back(e);
  }
  *e0 = g_prof.pool[at];
  *e1 = g_prof.pool[at + 1];
  g_prof.kind.push_back(kind);
  return true;
}

}  // namespace aplicur

using namespace aplicur;

extern "C" {

int aplicur_prof_products(int32_t enable) {
  std::lock_guard<std::mutex> g(g_prof.mu);
  if (enable) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
      set_last_error("hipGetDevice failed");
      return APLICUR_E_HIP;
    }
    if (dev != g_prof.device && !g_prof.kind.empty()) {
      set_last_error("read the recorded launches before switching device");
      return APLICUR_E_INVALID;
    }
    if (dev != g_prof.device) {
      for (hipEvent_t e : g_prof.pool) (void)hipEventDestroy(e);
      g_prof.pool.clear();
    }
    g_prof.device = dev;
  }
  g_prof.on = enable != 0;
  return APLICUR_OK;
}

int aplicur_prof_read(int64_t* launches, double* total_us, int64_t* untimed) {
  std::lock_guard<std::mutex> g(g_prof.mu);
  if (!launches || !total_us || !untimed) {
    set_last_error("bad argument");
    return APLICUR_E_INVALID;
  }
  for (int k = 0; k < kProfKinds; ++k) {
    launches[k] = 0;
    total_us[k] = 0.0;
    untimed[k] = g_prof.untimed[k];
  }
  int rc = APLICUR_OK;
  if (!g_prof.kind.empty()) {
    if (hipEventSynchronize(g_prof.pool[2 * g_prof.kind.size() - 1]) != hipSuccess) rc = APLICUR_E_HIP;
    for (size_t i = 0; i < g_prof.kind.size() && rc == APLICUR_OK; ++i) {
      float ms = 0.f;
      if (hipEventSynchronize(g_prof.pool[2 * i + 1]) != hipSuccess ||
          hipEventElapsedTime(&ms, g_prof.pool[2 * i], g_prof.pool[2 * i + 1]) != hipSuccess) {
        rc = APLICUR_E_HIP;
        break;
      }
      launches[g_prof.kind[i]] += 1;
      total_us[g_prof.kind[i]] += 1e3 * (double)ms;
    }
  }
  g_prof.kind.clear();
  for (auto& u : g_prof.untimed) u = 0;
  if (rc != APLICUR_OK) set_last_error("reading the product-kernel events failed");
  return rc;
}

}  // extern "C"
