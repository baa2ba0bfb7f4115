// IMEX step (Sec. 4.2): implicit collision, explicit streaming and source.  Isotropic: the
// same persistent kernel as the explicit step with the closed-form per-cell solve of
// (a I - c K~) psi' = b for the rank-one isotropic kernel K~ = w / (4 pi).  Moment-projected
// scattering: the per-cell diagonal and the final combine around the two moment products.
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

// Moment-form implicit collisions (eq. SNEqns2 inside the IMEX step of Sec. 4.2).  With
// M O = I the per-cell inverse of a_i I - b_i O Sigma M is (1/a_i)[I + O D_i M], D_i =
// diag(b_i Sigma_l / (a_i - b_i Sigma_l)), a_i = 1 + dt alpha_t sigma_t,i, b_i = dt alpha_s
// sigma_s,i.  The second moment product carries Sigma, so the moments U = M r between the two
// products are scaled by b_i / (a_i - b_i Sigma_l); one block per cell row, grid-stride.
template <typename T>
__global__ __launch_bounds__(256) void k_imex_moment_scale(T* __restrict__ U,
                                                           const T* __restrict__ sigma_t,
                                                           const T* __restrict__ sigma_s, T dt,
                                                           T alpha_t, T alpha_s,
                                                           const T* __restrict__ msig,
                                                           int64_t nc, int32_t mid) {
    for (int64_t c = blockIdx.x; c < nc; c += gridDim.x) {
        const T a = T(1) + dt * alpha_t * sigma_t[c];
        const T b = dt * alpha_s * sigma_s[c];
        T* row = U + c * mid;
        for (int32_t j = (int32_t)threadIdx.x; j < mid; j += 256) row[j] *= b / (a - b * msig[j]);
    }
}

// psi <- (r + S) / a_i in place: r is the collision-free explicit step, S = O D M r.  With
// c = dt alpha_t sigma_t the division by a_i = 1 + c is taken as x - x c / (1 + c), so that the
// rounding of 1 + c (half an ulp of 1, the same on every step) does not scale the state.
template <typename T>
__global__ __launch_bounds__(256) void k_imex_combine(T* __restrict__ psi, const T* __restrict__ S,
                                                      const T* __restrict__ sigma_t, T dt,
                                                      T alpha_t, int64_t nc, int32_t nq) {
    for (int64_t c = blockIdx.x; c < nc; c += gridDim.x) {
        const T cabs = dt * alpha_t * sigma_t[c];
        const T y = cabs / (T(1) + cabs);
        T* row = psi + c * nq;
        const T* srow = S + c * nq;
        for (int32_t q = (int32_t)threadIdx.x; q < nq; q += 256) {
            const T x = row[q] + srow[q];
            row[q] = x - x * y;
        }
    }
}

// FP32 rows of a multiple of 4 ordinates: 16-byte accesses, S read and psi written with
// the streaming bit (each is touched once here).
__global__ __launch_bounds__(256) void k_imex_combine4(f32x4* __restrict__ psi,
                                                       const f32x4* __restrict__ S,
                                                       const float* __restrict__ sigma_t,
                                                       float dt, float alpha_t, int64_t nc,
                                                       int32_t nq4) {
    for (int64_t c = blockIdx.x; c < nc; c += gridDim.x) {
        const float cabs = dt * alpha_t * sigma_t[c];
        const float y = cabs / (1.0f + cabs);
        f32x4* row = psi + c * nq4;
        const f32x4* srow = S + c * nq4;
        for (int32_t q = (int32_t)threadIdx.x; q < nq4; q += 256) {
            const f32x4 x = row[q] + __builtin_nontemporal_load(&srow[q]);
            __builtin_nontemporal_store(x - x * y, &row[q]);
        }
    }
}

// FP32 moment rows of a multiple of 4: 16-byte accesses.
__global__ __launch_bounds__(256) void k_imex_moment_scale4(f32x4* __restrict__ U,
                                                            const float* __restrict__ sigma_t,
                                                            const float* __restrict__ sigma_s,
                                                            float dt, float alpha_t,
                                                            float alpha_s,
                                                            const f32x4* __restrict__ msig,
                                                            int64_t nc, int32_t mid4) {
    for (int64_t c = blockIdx.x; c < nc; c += gridDim.x) {
        const float a = 1.0f + dt * alpha_t * sigma_t[c];
        const float b = dt * alpha_s * sigma_s[c];
        f32x4* row = U + c * mid4;
        for (int32_t j = (int32_t)threadIdx.x; j < mid4; j += 256) {
            const f32x4 sg = msig[j];
            f32x4 v = row[j];
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] *= b / (a - b * sg[k]);
            row[j] = v;
        }
    }
}

namespace {
constexpr int64_t kRowBlocksMax = 8192;
unsigned row_blocks(int64_t nc) { return (unsigned)std::min<int64_t>(nc, kRowBlocksMax); }
}  // namespace

template <typename T, typename A>
hipError_t launch_imex_moments_t(const A& a, T* U, const T* msig, int64_t nc, int32_t mid,
                                 int32_t nq, T* psi, const T* S, bool combine, hipStream_t st) {
    if (nc == 0) return hipSuccess;
    if (!combine)
        hipLaunchKernelGGL(k_imex_moment_scale<T>, dim3(row_blocks(nc)), dim3(256), 0, st, U,
                           a.sigma_t, a.sigma_s, a.dt, a.alpha_t, a.alpha_s, msig, nc, mid);
    else
        hipLaunchKernelGGL(k_imex_combine<T>, dim3(row_blocks(nc)), dim3(256), 0, st, psi, S,
                           a.sigma_t, a.dt, a.alpha_t, nc, nq);
    return hipGetLastError();
}

hipError_t launch_imex_moment_scale32(const StepArgs32& a, float* U, const float* msig,
                                      int64_t nc, int32_t mid, hipStream_t st) {
    // U sits 16-byte aligned in the workspace after S; msig is a device allocation
    if (nc > 0 && mid % 4 == 0 &&
        ((reinterpret_cast<uintptr_t>(U) | reinterpret_cast<uintptr_t>(msig)) & 15u) == 0) {
        hipLaunchKernelGGL(k_imex_moment_scale4, dim3(row_blocks(nc)), dim3(256), 0, st,
                           reinterpret_cast<f32x4*>(U), a.sigma_t, a.sigma_s, a.dt, a.alpha_t,
                           a.alpha_s, reinterpret_cast<const f32x4*>(msig), nc, mid / 4);
        return hipGetLastError();
    }
    return launch_imex_moments_t<float>(a, U, msig, nc, mid, 0, nullptr, nullptr, false, st);
}
hipError_t launch_imex_moment_scale64(const StepArgs64& a, double* U, const double* msig,
                                      int64_t nc, int32_t mid, hipStream_t st) {
    return launch_imex_moments_t<double>(a, U, msig, nc, mid, 0, nullptr, nullptr, false, st);
}
hipError_t launch_imex_combine32(const StepArgs32& a, float* psi, const float* S, int64_t nc,
                                 int32_t nq, hipStream_t st) {
    // state arrays are 16-byte aligned (checked by the library), so rows of 4k floats are too
    if (nc > 0 && nq % 4 == 0) {
        hipLaunchKernelGGL(k_imex_combine4, dim3(row_blocks(nc)), dim3(256), 0, st,
                           reinterpret_cast<f32x4*>(psi), reinterpret_cast<const f32x4*>(S),
                           a.sigma_t, a.dt, a.alpha_t, nc, nq / 4);
        return hipGetLastError();
    }
    return launch_imex_moments_t<float>(a, nullptr, nullptr, nc, 0, nq, psi, S, true, st);
}
hipError_t launch_imex_combine64(const StepArgs64& a, double* psi, const double* S, int64_t nc,
                                 int32_t nq, hipStream_t st) {
    return launch_imex_moments_t<double>(a, nullptr, nullptr, nc, 0, nq, psi, S, true, st);
}

}  // namespace snrt
