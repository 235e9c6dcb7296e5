// FP8 (e4m3) preconditioner chain: not built yet.
#include "common.h"

namespace kpcg {

hipError_t launch_precond_fp8(const Plan&, const float*, float*, const float*, bool, float,
                              hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace kpcg
