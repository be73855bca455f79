// Status strings, per-thread error detail and shared host helpers.
#include <stdarg.h>
#include <stdio.h>

#include "common.h"

namespace cld {

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
