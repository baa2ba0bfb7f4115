// The fused dense step with per-cell densities 1/rho (see sn_step_fused.h).
#include "sn_step_fused.h"

namespace snrt {

hipError_t launch_gemm_step_rho(const float* A, const uint16_t* Bhi, const uint16_t* Blo,
                                int64_t M, int32_t K, int32_t N, int products,
                                const int32_t* rexp, int32_t eb, const StepEpi& se,
                                hipStream_t st) {
    if (!se.a.inv_rho) return hipErrorInvalidValue;
    return fused::launch_gemm_step_t<true>(A, Bhi, Blo, M, K, N, products, rexp, eb, se, st);
}

}  // namespace snrt
