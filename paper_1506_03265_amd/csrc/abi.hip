// Status strings, per-thread error detail and shared host helpers.
#include <stdarg.h>
#include <stdio.h>

#include <atomic>
#include <mutex>
#include <vector>

#include "common.h"

namespace cld {

// Pinned host buffers for the small device-to-host readbacks of the host
// loops.  A call takes one for its duration and gives it back, so the pool
// grows only to the largest number of calls in flight at once and every
// buffer is reused (no allocation per call or per thread).
namespace {
std::mutex g_pinned_mu;
std::vector<void *> g_pinned_free;
std::atomic<int64_t> g_pinned_bytes{0};
}  // namespace

void *pinned_acquire(size_t bytes) {
  if (bytes > kPinnedBytes) return nullptr;
  {
    std::lock_guard<std::mutex> lk(g_pinned_mu);
    if (!g_pinned_free.empty()) {
      void *p = g_pinned_free.back();
      g_pinned_free.pop_back();
      return p;
    }
  }
  void *p = nullptr;
  // mapped and coherent: the host loops also poll words that kernels store into them
  if (hipHostMalloc(&p, kPinnedBytes, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) return nullptr;
  g_pinned_bytes += (int64_t)kPinnedBytes;
  return p;
}

void pinned_release(void *p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_pinned_mu);
  g_pinned_free.push_back(p);
}

static thread_local char t_err[512] = "";

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(t_err, sizeof t_err, fmt, ap);
  va_end(ap);
}

int hip_fail(hipError_t e, const char *what) {
  set_error("%s: %s", what, hipGetErrorString(e));
  return CLDIAM_EHIP;
}

int cooperative_blocks(const void *kernel, int threads, int max_per_cu, int *blocks) {
  *blocks = 0;
  int dev = 0, coop = 0, cus = 0, per_cu = 0;
  CLD_HIP(hipGetDevice(&dev));
  CLD_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
  CLD_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  if (!coop) return CLDIAM_OK;
  CLD_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0));
  if (per_cu > max_per_cu) per_cu = max_per_cu;
  *blocks = per_cu * cus;
  return CLDIAM_OK;
}

}  // namespace cld

extern "C" const char *cldiam_strerror(int status) {
  switch (status) {
    case CLDIAM_OK: return "ok";
    case CLDIAM_EINVAL: return "invalid argument";
    case CLDIAM_ENOMEM: return "workspace too small";
    case CLDIAM_EOVERFLOW: return "overflow";
    case CLDIAM_EHIP: return "HIP runtime error";
    case CLDIAM_ESTAGES: return "too many stages";
    case CLDIAM_ETIMEOUT: return "device wait timed out";
    default: return "unknown status";
  }
}

extern "C" const char *cldiam_last_error(void) { return cld::t_err; }

extern "C" const char *cldiam_version(void) { return "cldiam 0.1 gfx950"; }

extern "C" int64_t cldiam_pinned_host_bytes(void) { return cld::g_pinned_bytes.load(); }
