// Adjoint step (FP32 product path, the FP32 path with FP64 gradient accumulators, and the
// FP64 parity template).
#include "sn_step_kernels.h"

namespace snrt {

hipError_t launch_adjoint32(const snrt_mesh& m, const snrt_quad& q, const StepArgs32& a,
                            const float* psi_n, const float* lam_np1, float* lam_n, float* g_t,
                            float* g_s, float* g_r, const float* G, hipStream_t st) {
    return launch_adjoint_t<float>(m.geom32, m, q.tab32, q.nq, a, psi_n, lam_np1, lam_n, g_t,
                                   g_s, g_r, G, st);
}

hipError_t launch_adjoint32_acc64(const snrt_mesh& m, const snrt_quad& q, const StepArgs32& a,
                                  const float* psi_n, const float* lam_np1, float* lam_n,
                                  double* g_t, double* g_s, double* g_r, const float* G,
                                  hipStream_t st, const DoseAdj& da) {
    return launch_adjoint_t<float, double>(m.geom32, m, q.tab32, q.nq, a, psi_n, lam_np1, lam_n,
                                           g_t, g_s, g_r, G, st, da);
}

hipError_t launch_adjoint64(const snrt_mesh& m, const snrt_quad& q, const StepArgs64& a,
                            const double* psi_n, const double* lam_np1, double* lam_n,
                            double* g_t, double* g_s, double* g_r, const double* G,
                            hipStream_t st) {
    return launch_adjoint_t<double>(m.geom64, m, q.tab64, q.nq, a, psi_n, lam_np1, lam_n, g_t,
                                    g_s, g_r, G, st);
}

}  // namespace snrt
