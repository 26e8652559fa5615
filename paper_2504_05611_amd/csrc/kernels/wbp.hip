// Weighted (neural) min-sum BP: forward with checkpoints and hand-written backward.
#include <hip/hip_runtime.h>

#include "../host/device.h"

namespace tmcs {

size_t wbp_workspace_bytes(const Dem& d, int T, uint64_t n_shots) { (void)d; (void)T; (void)n_shots; return 0; }

tmcs_status wbp_forward_run(const Dem&, const float*, int, const uint64_t*, uint64_t, float*, void*, size_t,
                            hipStream_t) {
  return fail(TMCS_EUNSUPPORTED, "weighted BP not built yet");
}

tmcs_status wbp_backward_run(const Dem&, const float*, int, const uint64_t*, uint64_t, const float*, float*,
                             const void*, size_t, hipStream_t) {
  return fail(TMCS_EUNSUPPORTED, "weighted BP not built yet");
}

}  // namespace tmcs
