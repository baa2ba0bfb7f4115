// Per-cell angular integrals and global reductions (FP64 accumulation), and row permutes.
//
//   scalar flux  phi_i = sum_q w_q psi_iq                         (Sec. 7.2)
//   mass         M = sum_i A_i phi_i                              (solver log, Sec. 5.1)
//   dose         D_i += coeff * (1/rho_i) * phi_i                 (Sec. 2, pseudo-time form)
//
// One wavefront per cell; lane l sums ordinates l, l+64, ... in FP64, then a butterfly
// reduction.  The mass is a deterministic two-pass tree: per-block partials, then one block
// folds them in a fixed order.
#include "snrt_internal.h"

namespace snrt {

namespace {

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// phi of cell c in FP64 (all lanes get the value)
__device__ __forceinline__ double cell_phi(const float* __restrict__ psi,
                                           const double* __restrict__ w, int64_t c, int32_t nq,
                                           int lane) {
    const float* row = psi + c * (int64_t)nq;
    double s = 0.0;
    for (int q = lane; q < nq; q += kWave) s += w[q] * (double)row[q];
    return wave_sum_d(s);
}

__global__ __launch_bounds__(kStepBlock) void k_mass_partial(const CellGeom64* __restrict__ geom,
                                                             const float* __restrict__ psi,
                                                             const double* __restrict__ w,
                                                             int64_t nc, int32_t nq,
                                                             double* __restrict__ partial)
{
    __shared__ double red[kCellsPerBlock];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
    const int64_t c = (int64_t)blockIdx.x * kCellsPerBlock + wave;
    double v = 0.0;
    if (c < nc) v = geom[c].area * cell_phi(psi, w, c, nq, lane);
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < kCellsPerBlock; ++i) s += red[i];
        partial[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(1024) void k_fold(const double* __restrict__ partial, int64_t n,
                                               double* __restrict__ out)
{
    __shared__ double red[1024];
    const int t = threadIdx.x;
    double s = 0.0;
    for (int64_t i = t; i < n; i += 1024) s += partial[i];
    red[t] = s;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    if (t == 0) *out = red[0];
}

__global__ __launch_bounds__(kStepBlock) void k_scalar_flux(const float* __restrict__ psi,
                                                            const double* __restrict__ w,
                                                            int64_t nc, int32_t nq,
                                                            float* __restrict__ phi)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
    const int64_t c = (int64_t)blockIdx.x * kCellsPerBlock + wave;
    if (c >= nc) return;
    const double s = cell_phi(psi, w, c, nq, lane);
    if (lane == 0) phi[c] = (float)s;
}

__global__ __launch_bounds__(kStepBlock) void k_dose(const float* __restrict__ psi,
                                                     const double* __restrict__ w,
                                                     const float* __restrict__ inv_rho,
                                                     double coeff, int64_t nc, int32_t nq,
                                                     double* __restrict__ dose)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
    const int64_t c = (int64_t)blockIdx.x * kCellsPerBlock + wave;
    if (c >= nc) return;
    const double s = cell_phi(psi, w, c, nq, lane);
    if (lane == 0) dose[c] += coeff * (inv_rho ? (double)inv_rho[c] : 1.0) * s;
}

// out[k] = in[src(k)] row copy in 4-byte words; to_user: out[perm[k]] = in[k]
__global__ __launch_bounds__(256) void k_permute(const uint32_t* __restrict__ in,
                                                 uint32_t* __restrict__ out,
                                                 const int64_t* __restrict__ perm, int64_t nc,
                                                 int64_t words, int to_user)
{
    const int64_t k = blockIdx.x;
    if (k >= nc) return;
    const int64_t src = to_user ? k : perm[k];
    const int64_t dst = to_user ? perm[k] : k;
    for (int64_t i = threadIdx.x; i < words; i += 256) out[dst * words + i] = in[src * words + i];
}

// lam[c][q] += coeff * w_q * inv_rho[c] * g_dose[c]: one wavefront per cell
__global__ __launch_bounds__(kStepBlock) void k_dose_adjoint(const double* __restrict__ w,
                                                             const float* __restrict__ inv_rho,
                                                             double coeff,
                                                             const double* __restrict__ g_dose,
                                                             float* __restrict__ lam, int64_t nc,
                                                             int32_t nq)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
    const int64_t c = (int64_t)blockIdx.x * kCellsPerBlock + wave;
    if (c >= nc) return;
    const double g = coeff * (inv_rho ? (double)inv_rho[c] : 1.0) * g_dose[c];
    float* row = lam + c * (int64_t)nq;
    for (int q = lane; q < nq; q += kWave) row[q] = (float)((double)row[q] + g * w[q]);
}

__global__ __launch_bounds__(256) void k_dose_density_grad(const double* __restrict__ dose,
                                                           const float* __restrict__ inv_rho,
                                                           const double* __restrict__ g_dose,
                                                           float* __restrict__ g_rho, int64_t nc)
{
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= nc) return;
    g_rho[c] = (float)((double)g_rho[c] - dose[c] * (inv_rho ? (double)inv_rho[c] : 1.0) * g_dose[c]);
}

inline unsigned blocks_for(int64_t nc) {
    return (unsigned)((nc + kCellsPerBlock - 1) / kCellsPerBlock);
}

}  // namespace

hipError_t launch_mass(const snrt_mesh& m, const snrt_quad& q, const float* psi, double* out,
                       hipStream_t st) {
    if (m.nc == 0) {   // a fill kernel, not a memset node: callers may capture this in a graph
        hipLaunchKernelGGL(k_fold, dim3(1), dim3(1024), 0, st, m.d_partial, (int64_t)0, out);
        return hipGetLastError();
    }
    const unsigned nb = blocks_for(m.nc);
    hipLaunchKernelGGL(k_mass_partial, dim3(nb), dim3(kStepBlock), 0, st, m.geom64, psi,
                       q.tab64 + 2 * (int64_t)q.nq, m.nc, q.nq, m.d_partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fold, dim3(1), dim3(1024), 0, st, m.d_partial, (int64_t)nb, out);
    return hipGetLastError();
}

hipError_t launch_scalar_flux(const snrt_mesh& m, const snrt_quad& q, const float* psi,
                              float* phi, hipStream_t st) {
    if (m.nc == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scalar_flux, dim3(blocks_for(m.nc)), dim3(kStepBlock), 0, st, psi,
                       q.tab64 + 2 * (int64_t)q.nq, m.nc, q.nq, phi);
    return hipGetLastError();
}

hipError_t launch_dose(const snrt_mesh& m, const snrt_quad& q, const float* psi,
                       const float* inv_rho, double coeff, double* dose, hipStream_t st) {
    if (m.nc == 0) return hipSuccess;
    hipLaunchKernelGGL(k_dose, dim3(blocks_for(m.nc)), dim3(kStepBlock), 0, st, psi,
                       q.tab64 + 2 * (int64_t)q.nq, inv_rho, coeff, m.nc, q.nq, dose);
    return hipGetLastError();
}

hipError_t launch_permute(const snrt_mesh& m, int to_user, const void* in, void* out,
                          int64_t row_bytes, hipStream_t st) {
    if (m.nc == 0) return hipSuccess;
    hipLaunchKernelGGL(k_permute, dim3((unsigned)m.nc), dim3(256), 0, st,
                       static_cast<const uint32_t*>(in), static_cast<uint32_t*>(out),
                       m.d_to_user, m.nc, row_bytes / 4, to_user);
    return hipGetLastError();
}

hipError_t launch_dose_adjoint(const snrt_mesh& m, const snrt_quad& q, const float* inv_rho,
                               double coeff, const double* g_dose, float* lam, hipStream_t st) {
    if (m.nc == 0) return hipSuccess;
    hipLaunchKernelGGL(k_dose_adjoint, dim3(blocks_for(m.nc)), dim3(kStepBlock), 0, st,
                       q.tab64 + 2 * (int64_t)q.nq, inv_rho, coeff, g_dose, lam, m.nc, q.nq);
    return hipGetLastError();
}

hipError_t launch_dose_density_grad(const snrt_mesh& m, const double* dose, const float* inv_rho,
                                    const double* g_dose, float* g_rho, hipStream_t st) {
    if (m.nc == 0) return hipSuccess;
    hipLaunchKernelGGL(k_dose_density_grad, dim3((unsigned)((m.nc + 255) / 256)), dim3(256), 0, st,
                       dose, inv_rho, g_dose, g_rho, m.nc);
    return hipGetLastError();
}

}  // namespace snrt
