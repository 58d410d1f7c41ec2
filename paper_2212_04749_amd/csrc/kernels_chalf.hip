// complex-half kernels (FP16 storage, per-instance power-of-two exponent,
// FP16 MFMA with FP32 accumulation).
#include <hip/hip_runtime.h>

#include "desc.h"
#include "kernels.h"

namespace matnc {

bool chalf_available() { return false; }

int mfma_h_config_count() { return 0; }
bool mfma_h_config_fits(int, int, int, int) { return false; }
hipError_t launch_mfma_h(const NodeDesc&, int, uint64_t, const int64_t*, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_slice_sum_h(const OpDesc&, uint64_t, const int64_t*, int, int64_t, int, double*, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace matnc
