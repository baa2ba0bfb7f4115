// FP32 forward step: instantiation of the step kernels for the product path.
#include "sn_step_kernels.h"

namespace snrt {

hipError_t launch_step32(const snrt_mesh& m, const snrt_quad& q, const StepArgs32& a,
                         const float* psi_in, float* psi_out, const float* S, hipStream_t st) {
    return launch_step_t<float>(m.geom32, m, q.tab32, q.nq, a, psi_in, psi_out, S, st);
}

}  // namespace snrt
