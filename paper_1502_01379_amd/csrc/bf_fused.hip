// Fused MFMA passes (placeholder until the kernels land).
#include <hip/hip_runtime.h>

#include "bf_internal.h"

namespace bfly {

struct FusedPass {};

bool fused_supported(const bf_shape &, bf_precision) { return false; }
bf_status fused_build(bf_plan *, const bf_factors_host *) { return BF_ERR_UNSUPPORTED; }
hipError_t fused_run(bf_plan *, bool, const void *, void *, int64_t, int64_t, void *, void *,
                     hipStream_t) {
  return hipErrorNotSupported;
}
void fused_free(FusedPass *fp) { delete fp; }

}  // namespace bfly
