// The mode-space IMEX combine in one launch with its product (kernel templates in
// sn_step_fused.h).
#include "sn_step_fused.h"

namespace snrt {

hipError_t launch_gemm_combine(const float* A, const uint16_t* Bhi, const uint16_t* Blo,
                               int64_t M, int32_t K, int32_t N, int products,
                               const int32_t* rexp, int32_t eb, const CombineEpi& ce,
                               hipStream_t st) {
    return fused::launch_gemm_combine_impl(A, Bhi, Blo, M, K, N, products, rexp, eb, ce, st);
}

}  // namespace snrt
