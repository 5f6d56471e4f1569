// Fused single-pass Taylor-4 step.  (Work in progress: not yet enabled.)
#include <hip/hip_runtime.h>

#include "fused.h"

bool fused_supported(const abc_params& p, std::string* why) {
  (void)p;
  if (why) *why = "not available in this build";
  return false;
}

abc_status fused_prepare(const abc_params&, abc_launch&, std::vector<void*>*, size_t*, std::string& err) {
  err = "fused path not available";
  return ABC_ENOTSUP;
}

hipError_t launch_step_fused(const abc_launch&, const abc_scratch&, void*, double2*, const void*, int, hipStream_t) {
  return hipErrorNotSupported;
}
