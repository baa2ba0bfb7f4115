// IMEX step (Sec. 4.2): implicit isotropic collision, explicit streaming and source.  The
// same persistent kernel as the explicit step with the closed-form per-cell solve of
// (a I - c K~) psi' = b for the rank-one isotropic kernel K~ = w / (4 pi).
#include "sn_step_kernels.h"

namespace snrt {

hipError_t launch_imex32(const snrt_mesh& m, const snrt_quad& q, const StepArgs32& a,
                         const float* psi_in, float* psi_out, hipStream_t st) {
    return launch_imex_t<float>(m.geom32, m, q.tab32, q.nq, a, psi_in, psi_out, st);
}

hipError_t launch_imex64(const snrt_mesh& m, const snrt_quad& q, const StepArgs64& a,
                         const double* psi_in, double* psi_out, hipStream_t st) {
    return launch_imex_t<double>(m.geom64, m, q.tab64, q.nq, a, psi_in, psi_out, st);
}

}  // namespace snrt
