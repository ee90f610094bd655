// Batched KL as one contraction over the log-kernel (placeholder until the
// MFMA kernel lands: reports "not supported").
#include "dd_internal.h"

namespace dd {

size_t batch_kl_workspace(GemmView, int32_t) { return 0; }

hipError_t launch_batch_kl(DenseView, GemmView, const int32_t*, int32_t, void*, size_t, float*,
                           hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace dd
