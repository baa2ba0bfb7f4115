// The unrolled P_N step kernels of degree 13 (FP32), in a translation unit of its own: the
// operator table unrolls to about 12 000 coefficient applications per z-parity subsystem,
// and compiling it beside the other degrees would serialise the build.  The matrix-core form
// (k_pn_mfma: dense class blocks on the matrix cores) runs by default; SNRT_PN_MFMA=0
// selects the all-vector kernel.
#include "sn_pn_kernels.h"

namespace snrt {

hipError_t launch_pn_fused_high32(const snrt_mesh& m, const snrt_pn& p, const StepArgs32& a,
                                  const float* u, float* out, hipStream_t st) {
    constexpr int N = pn::kFusedHighDegree;
    if (p.degree != N) return hipErrorInvalidValue;
    if (tune().pn_mfma && p.wa16)
        return m.mf == 3 ? launch_mfma_t<N, 3>(m, p, a, u, out, st)
                         : launch_mfma_t<N, 4>(m, p, a, u, out, st);
    return m.mf == 3 ? launch_fused_t<N, 3, float>(m, p, a, p.w32, p.sig32, u, out, st)
                     : launch_fused_t<N, 4, float>(m, p, a, p.w32, p.sig32, u, out, st);
}

}  // namespace snrt
