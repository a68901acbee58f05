// FP32 cell-relative packet tracking (built in a later step).
#include <hip/hip_runtime.h>

#include "mcrt_internal.h"

namespace mcrt {
int launch_trace_fp32(mcrt_ctx* ctx, const TraceArgs&, hipStream_t) {
  set_error(ctx, "FP32 tracking is not available in this build");
  return MCRT_E_ARG;
}
}  // namespace mcrt
