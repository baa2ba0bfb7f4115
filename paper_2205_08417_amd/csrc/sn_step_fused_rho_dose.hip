// The one-launch dense step with densities and the dose of its input (kernel templates in sn_step_fused.h).
#include "sn_step_fused.h"

namespace snrt {
namespace fused {

template hipError_t launch_gemm_step_t<true, true>(const float*, const uint16_t*,
                                                  const uint16_t*, int64_t, int32_t, int32_t,
                                                  int, const int32_t*, int32_t, const StepEpi&,
                                                  hipStream_t);

}  // namespace fused
}  // namespace snrt
