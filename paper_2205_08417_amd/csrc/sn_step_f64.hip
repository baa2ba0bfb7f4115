// FP64 forward step: the parity template of the FP32 kernels (same code, double).
#include "sn_step_kernels.h"

namespace snrt {

hipError_t launch_step64(const snrt_mesh& m, const snrt_quad& q, const StepArgs64& a,
                         const double* psi_in, double* psi_out, const double* S,
                         hipStream_t st) {
    return launch_step_t<double>(m.geom64, m, q.tab64, q.nq, a, psi_in, psi_out, S, st);
}

hipError_t launch_free_step64(const snrt_mesh& m, const snrt_quad& q, const StepArgs64& a,
                              const double* psi_in, double* psi_out, hipStream_t st) {
    return launch_step_t<double>(m.geom64, m, q.tab64, q.nq, a, psi_in, psi_out, nullptr, st,
                                 nullptr, nullptr, true);
}

}  // namespace snrt
