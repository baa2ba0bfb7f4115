// Per-cell angular integrals and global reductions (FP64 accumulation), and row permutes.
//
//   scalar flux  phi_i = sum_q w_q psi_iq                         (Sec. 7.2)
//   mass         M = sum_i A_i phi_i                              (solver log, Sec. 5.1)
//   dose         D_i += coeff * (1/rho_i) * phi_i                 (Sec. 2, pseudo-time form)
//
// Persistent wavefronts stride over the cells; lane l owns the V contiguous ordinates
// [l*V, l*V+V) of a row (16-byte loads) and keeps their FP64 weights in registers, sums its
// slice in FP64 and the wave adds the 64 partial sums with a butterfly.  The next row is
// loaded while the current one is reduced.  The mass is a deterministic two-pass tree: one
// partial per wave (a fixed set of cells in a fixed order), then one block folds them.
#include "sn_step_kernels.h"

namespace snrt {

namespace {

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

constexpr int kReduceBlocksPerCu = 4;

template <int V, bool EXACT>
struct RowPhi {
    double wv[V];
    int q0;
    int32_t nq;
    __device__ __forceinline__ RowPhi(const double* __restrict__ w, int32_t nq_, int lane)
        : q0(lane * V), nq(nq_) {
#pragma unroll
        for (int k = 0; k < V; ++k) wv[k] = (q0 + k < nq) ? w[q0 + k] : 0.0;
    }
    __device__ __forceinline__ void load(const float* __restrict__ psi, int64_t c, float (&r)[V]) const {
        load_slice<V, EXACT>(psi + c * (int64_t)nq, q0, nq, r);
    }
    __device__ __forceinline__ double sum(const float (&r)[V]) const {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < V; ++k) s += wv[k] * (double)r[k];
        return wave_sum_d(s);
    }
};

// Visit every cell c of this wave's share in increasing order with phi(c); the row of the
// next cell is in flight while the current one is reduced.
template <int V, bool EXACT, typename F>
__device__ __forceinline__ void for_each_phi(const float* __restrict__ psi,
                                             const double* __restrict__ w, int64_t nc,
                                             int32_t nq, F&& visit) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x / kWave);
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
    const RowPhi<V, EXACT> rp(w, nq, lane);
    int64_t c = gw;
    if (c >= nc) return;
    float cur[V], nxt[V];
    rp.load(psi, c, cur);
    for (;;) {
        const int64_t cn = c + nw;
        if (cn < nc) rp.load(psi, cn, nxt);
        visit(c, rp.sum(cur));
        if (cn >= nc) break;
        __builtin_memcpy(cur, nxt, sizeof(cur));
        c = cn;
    }
}

template <int V, bool EXACT>
__global__ __launch_bounds__(kStepBlock) void k_mass_partial(const CellGeom64* __restrict__ geom,
                                                             const float* __restrict__ psi,
                                                             const double* __restrict__ w,
                                                             int64_t nc, int32_t nq,
                                                             double* __restrict__ partial)
{
    double acc = 0.0;
    for_each_phi<V, EXACT>(psi, w, nc, nq, [&](int64_t c, double phi) {
        acc += geom[c].area * phi;
    });
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) partial[gw] = acc;
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

template <int V, bool EXACT>
__global__ __launch_bounds__(kStepBlock) void k_scalar_flux(const float* __restrict__ psi,
                                                            const double* __restrict__ w,
                                                            int64_t nc, int32_t nq,
                                                            float* __restrict__ phi)
{
    const bool lane0 = (threadIdx.x & (kWave - 1)) == 0;
    for_each_phi<V, EXACT>(psi, w, nc, nq, [&](int64_t c, double s) {
        if (lane0) phi[c] = (float)s;
    });
}

template <int V, bool EXACT>
__global__ __launch_bounds__(kStepBlock) void k_dose(const float* __restrict__ psi,
                                                     const double* __restrict__ w,
                                                     const float* __restrict__ inv_rho,
                                                     double coeff, int64_t nc, int32_t nq,
                                                     double* __restrict__ dose)
{
    const bool lane0 = (threadIdx.x & (kWave - 1)) == 0;
    for_each_phi<V, EXACT>(psi, w, nc, nq, [&](int64_t c, double s) {
        if (lane0) dose[c] += coeff * (inv_rho ? (double)inv_rho[c] : 1.0) * s;
    });
}

// dose[c] += coeff * inv_rho[c] * sum_k part[c * nch + k]: the fused step's per-item sums
// of the state entering the step, folded in a fixed order (one thread per cell)
__global__ __launch_bounds__(256) void k_dose_fold(const double* __restrict__ part, int32_t nch,
                                                   const float* __restrict__ inv_rho,
                                                   double coeff, int64_t nc,
                                                   double* __restrict__ dose)
{
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= nc) return;
    double s = 0.0;
    for (int32_t k = 0; k < nch; ++k) s += part[c * nch + k];
    dose[c] += coeff * (inv_rho ? (double)inv_rho[c] : 1.0) * s;
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

// lam[c][q] += coeff * w_q * inv_rho[c] * g_dose[c]: persistent waves, V ordinates per lane
template <int V, bool EXACT>
__global__ __launch_bounds__(kStepBlock) void k_dose_adjoint(const double* __restrict__ w,
                                                             const float* __restrict__ inv_rho,
                                                             double coeff,
                                                             const double* __restrict__ g_dose,
                                                             float* __restrict__ lam, int64_t nc,
                                                             int32_t nq)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x / kWave);
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
    const int q0 = lane * V;
    double wv[V];
#pragma unroll
    for (int k = 0; k < V; ++k) wv[k] = (q0 + k < nq) ? w[q0 + k] : 0.0;
    for (int64_t c = gw; c < nc; c += nw) {
        const double g = coeff * (inv_rho ? (double)inv_rho[c] : 1.0) * g_dose[c];
        float* row = lam + c * (int64_t)nq;
        float r[V];
        load_slice<V, EXACT>(row, q0, nq, r);
#pragma unroll
        for (int k = 0; k < V; ++k) r[k] = (float)__builtin_fma(g, wv[k], (double)r[k]);
        store_slice<V, EXACT>(row, q0, nq, r, false);
    }
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

__global__ __launch_bounds__(256) void k_dose_density_grad64(const double* __restrict__ dose,
                                                             const float* __restrict__ inv_rho,
                                                             const double* __restrict__ g_dose,
                                                             double* __restrict__ g_rho, int64_t nc)
{
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= nc) return;
    g_rho[c] -= dose[c] * (inv_rho ? (double)inv_rho[c] : 1.0) * g_dose[c];
}

inline unsigned blocks_for(int64_t nc) {
    return (unsigned)((nc + kCellsPerBlock - 1) / kCellsPerBlock);
}

// Persistent reduction grid: at most kReduceBlocksPerCu blocks per CU and never more waves than
// the mesh holds partial slots for.
inline unsigned reduce_blocks(const snrt_mesh& m) {
    int64_t b = (int64_t)m.num_cu * kReduceBlocksPerCu;
    const int64_t cap = m.n_partial / kCellsPerBlock;
    if (b > cap) b = cap;
    const int64_t want = (m.nc + kCellsPerBlock - 1) / kCellsPerBlock;
    if (b > want) b = want;
    return (unsigned)(b < 1 ? 1 : b);
}

// Streaming copy for bandwidth measurement: 16-byte nontemporal loads and stores, four per
// lane per grid-stride round (an attainable read+write rate for a state-sized buffer).
constexpr int kCopyUnroll = 4;

__global__ __launch_bounds__(256) void k_stream_copy(const f32x4* __restrict__ src,
                                                     f32x4* __restrict__ dst, int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * 256 * kCopyUnroll;
    for (int64_t base = (int64_t)blockIdx.x * 256 * kCopyUnroll + threadIdx.x; base < n16;
         base += stride) {
        f32x4 v[kCopyUnroll];
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u) {
            const int64_t i = base + (int64_t)u * 256;
            if (i < n16) v[u] = __builtin_nontemporal_load(&src[i]);
        }
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u) {
            const int64_t i = base + (int64_t)u * 256;
            if (i < n16) __builtin_nontemporal_store(v[u], &dst[i]);
        }
    }
}

}  // namespace

hipError_t launch_mass(const snrt_mesh& m, const snrt_quad& q, const float* psi, double* out,
                       hipStream_t st) {
    if (m.nc == 0) {   // a fill kernel, not a memset node: callers may capture this in a graph
        hipLaunchKernelGGL(k_fold, dim3(1), dim3(1024), 0, st, m.d_partial, (int64_t)0, out);
        return hipGetLastError();
    }
    const unsigned nb = reduce_blocks(m);
    hipError_t e = dispatch_v<float>(q.nq, [&](auto vc, auto ex) {
        constexpr int V = decltype(vc)::value;
        constexpr bool E = decltype(ex)::value;
        hipLaunchKernelGGL((k_mass_partial<V, E>), dim3(nb), dim3(kStepBlock), 0, st, m.geom64,
                           psi, q.tab64 + 2 * (int64_t)q.nq, m.nc, q.nq, m.d_partial);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fold, dim3(1), dim3(1024), 0, st, m.d_partial,
                       (int64_t)nb * kCellsPerBlock, out);
    return hipGetLastError();
}

hipError_t launch_scalar_flux(const snrt_mesh& m, const snrt_quad& q, const float* psi,
                              float* phi, hipStream_t st) {
    if (m.nc == 0) return hipSuccess;
    return dispatch_v<float>(q.nq, [&](auto vc, auto ex) {
        constexpr int V = decltype(vc)::value;
        constexpr bool E = decltype(ex)::value;
        hipLaunchKernelGGL((k_scalar_flux<V, E>), dim3(reduce_blocks(m)), dim3(kStepBlock), 0,
                           st, psi, q.tab64 + 2 * (int64_t)q.nq, m.nc, q.nq, phi);
        return hipGetLastError();
    });
}

hipError_t launch_dose(const snrt_mesh& m, const snrt_quad& q, const float* psi,
                       const float* inv_rho, double coeff, double* dose, hipStream_t st) {
    if (m.nc == 0) return hipSuccess;
    return dispatch_v<float>(q.nq, [&](auto vc, auto ex) {
        constexpr int V = decltype(vc)::value;
        constexpr bool E = decltype(ex)::value;
        hipLaunchKernelGGL((k_dose<V, E>), dim3(reduce_blocks(m)), dim3(kStepBlock), 0, st, psi,
                           q.tab64 + 2 * (int64_t)q.nq, inv_rho, coeff, m.nc, q.nq, dose);
        return hipGetLastError();
    });
}

hipError_t launch_dose_fold(const snrt_mesh& m, const double* part, int32_t nch,
                            const float* inv_rho, double coeff, double* dose, hipStream_t st) {
    if (m.nc == 0) return hipSuccess;
    hipLaunchKernelGGL(k_dose_fold, dim3((unsigned)((m.nc + 255) / 256)), dim3(256), 0, st, part,
                       nch, inv_rho, coeff, m.nc, dose);
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
    return dispatch_v<float>(q.nq, [&](auto vc, auto ex) {
        constexpr int V = decltype(vc)::value;
        constexpr bool E = decltype(ex)::value;
        hipLaunchKernelGGL((k_dose_adjoint<V, E>), dim3(reduce_blocks(m)), dim3(kStepBlock), 0,
                           st, q.tab64 + 2 * (int64_t)q.nq, inv_rho, coeff, g_dose, lam, m.nc,
                           q.nq);
        return hipGetLastError();
    });
}

hipError_t launch_dose_density_grad(const snrt_mesh& m, const double* dose, const float* inv_rho,
                                    const double* g_dose, float* g_rho, hipStream_t st) {
    if (m.nc == 0) return hipSuccess;
    hipLaunchKernelGGL(k_dose_density_grad, dim3((unsigned)((m.nc + 255) / 256)), dim3(256), 0, st,
                       dose, inv_rho, g_dose, g_rho, m.nc);
    return hipGetLastError();
}

hipError_t launch_dose_density_grad64(const snrt_mesh& m, const double* dose,
                                      const float* inv_rho, const double* g_dose, double* g_rho,
                                      hipStream_t st) {
    if (m.nc == 0) return hipSuccess;
    hipLaunchKernelGGL(k_dose_density_grad64, dim3((unsigned)((m.nc + 255) / 256)), dim3(256), 0,
                       st, dose, inv_rho, g_dose, g_rho, m.nc);
    return hipGetLastError();
}

hipError_t launch_stream_copy(const void* src, void* dst, int64_t bytes, hipStream_t st) {
    const int64_t n16 = bytes / 16;
    if (n16 == 0) return hipSuccess;
    // 32 blocks per CU were measured as fast as one block per 1024 vectors
    const int64_t want = (n16 + 256 * kCopyUnroll - 1) / (256 * kCopyUnroll);
    const unsigned nb = (unsigned)std::min<int64_t>(want, 8192);
    hipLaunchKernelGGL(k_stream_copy, dim3(nb), dim3(256), 0, st,
                       static_cast<const f32x4*>(src), static_cast<f32x4*>(dst), n16);
    return hipGetLastError();
}

}  // namespace snrt
