// The transposed dense step in one launch with its product (kernel templates in
// sn_step_fused.h), and the fold of its per-piece gradient sums into the per-cell gradients.
#include "sn_step_fused.h"

namespace snrt {

hipError_t launch_gemm_adjoint(const float* A, const uint16_t* Bhi, const uint16_t* Blo,
                               int64_t M, int32_t K, int32_t N, int products,
                               const int32_t* rexp, int32_t eb, const AdjEpi& ae,
                               hipStream_t st) {
    return ae.da.g_dose
               ? fused::launch_gemm_adjoint_impl<true>(A, Bhi, Blo, M, K, N, products, rexp, eb,
                                                       ae, st)
               : fused::launch_gemm_adjoint_impl<false>(A, Bhi, Blo, M, K, N, products, rexp,
                                                        eb, ae, st);
}

namespace {

// one thread per cell: the pieces of the cell's row summed in order, scaled as the
// transposed-step kernel scales its whole-row sums
template <typename GT>
__global__ __launch_bounds__(256) void k_adjoint_fold(int64_t nc, int32_t np, StepArgs32 a,
                                                      const float* __restrict__ part,
                                                      GT* __restrict__ g_t, GT* __restrict__ g_s,
                                                      GT* __restrict__ g_r)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const float* p = part + c * np * 3;
    float st = 0.0f, ss = 0.0f, sr = 0.0f;
    for (int k = 0; k < np; ++k) {
        st += p[3 * k];
        ss += p[3 * k + 1];
        sr += p[3 * k + 2];
    }
    const float irho = a.inv_rho ? a.inv_rho[c] : 1.0f;
    if (g_t) g_t[c] = g_t[c] + (GT)(-a.dt * a.alpha_t * st);
    if (g_s) g_s[c] = g_s[c] + (GT)(a.dt * a.alpha_s * ss);
    if (g_r) g_r[c] = g_r[c] + (GT)(a.dt * irho * irho * sr);
}

template <typename GT>
hipError_t fold(int64_t nc, int32_t np, const StepArgs32& a, const float* part, GT* g_t,
                GT* g_s, GT* g_r, hipStream_t st) {
    if (nc == 0 || (!g_t && !g_s && !g_r)) return hipSuccess;
    if (np <= 0 || !part) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_adjoint_fold<GT>, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st,
                       nc, np, a, part, g_t, g_s, g_r);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_adjoint_fold32(int64_t nc, int32_t npieces, const StepArgs32& a,
                                 const float* part, float* g_t, float* g_s, float* g_r,
                                 hipStream_t st) {
    return fold(nc, npieces, a, part, g_t, g_s, g_r, st);
}

hipError_t launch_adjoint_fold64(int64_t nc, int32_t npieces, const StepArgs32& a,
                                 const float* part, double* g_t, double* g_s, double* g_r,
                                 hipStream_t st) {
    return fold(nc, npieces, a, part, g_t, g_s, g_r, st);
}

}  // namespace snrt
