// BF16 MFMA scattering product (placeholder until the gfx950 kernel lands).
#include "snrt_internal.h"

namespace snrt {

hipError_t launch_split_bf16(const float*, uint16_t*, uint16_t*, int32_t, hipStream_t) {
    return hipErrorNotSupported;
}

hipError_t launch_gemm_bf16(const float*, const uint16_t*, const uint16_t*, float*, int64_t,
                            int32_t, bool, hipStream_t) {
    return hipErrorNotSupported;
}

}  // namespace snrt
