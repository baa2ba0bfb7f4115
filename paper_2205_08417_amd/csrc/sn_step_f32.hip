// FP32 forward step: instantiation of the step kernels for the product path.
#include "sn_step_kernels.h"

namespace snrt {

hipError_t launch_step32(const snrt_mesh& m, const snrt_quad& q, const StepArgs32& a,
                         const float* psi_in, float* psi_out, const float* S, hipStream_t st,
                         double* dose_part) {
    return launch_step_t<float>(m.geom32, m, q.tab32, q.nq, a, psi_in, psi_out, S, st,
                                q.tab64 + 2 * (int64_t)q.nq, dose_part);
}

hipError_t launch_free_step32(const snrt_mesh& m, const snrt_quad& q, const StepArgs32& a,
                              const float* psi_in, float* psi_out, hipStream_t st) {
    return launch_step_t<float>(m.geom32, m, q.tab32, q.nq, a, psi_in, psi_out, nullptr, st,
                                nullptr, nullptr, true);
}

int32_t step_items_per_row(const snrt_quad& q, bool dense) {
    return dense ? 1 << dense_chunk_shift(q.nq) : 1;
}

}  // namespace snrt
