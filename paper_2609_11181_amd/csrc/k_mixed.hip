// Mixed batches of plans in one launch.
#include <hip/hip_runtime.h>

#include "smart_internal.h"

namespace smart {

int mixed_batch(smart_ctx ctx, int n_plans, const smart_plan* plans, const int* norms, void* const* outs,
                hipStream_t st) {
  (void)ctx; (void)n_plans; (void)plans; (void)norms; (void)outs; (void)st;
  set_error("mixed batches are not available in this build");
  return SMART_EUNSUPPORTED;
}

}  // namespace smart
