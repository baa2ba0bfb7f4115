// P_N step on gfx950: the degree dispatch, the chunked kernel for degrees without an
// unrolled one, the layout conversion and the library entry points of the kernels in
// sn_pn_kernels.h (the unrolled degree above the contiguous range is instantiated in
// sn_pn13.hip, a translation unit of its own).
#include "sn_pn_kernels.h"

namespace snrt {

namespace {

// Any degree: output moments in chunks of CH, the coefficients from the dense table
// W[m][nmp][4] (zero outside the patterns and in the padding).
template <int CH, int MF, typename T>
__global__ __launch_bounds__(256) void k_pn_generic(const typename GeomOf<T>::type* __restrict__ geom,
                                                    int32_t nc, int32_t ntiles, int32_t nm,
                                                    int32_t nmp, const T* __restrict__ W,
                                                    const T* __restrict__ sig,
                                                    typename ArgsOf<T>::type a,
                                                    const T* __restrict__ u, T* __restrict__ out,
                                                    uint32_t state_bytes) {
    const uint32_t kPlane = kTile * sizeof(T);
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int tile = (int)(blk * 4 + (threadIdx.x >> 6));
    const int c = tile * kTile + (int)(threadIdx.x & 63);
    if (tile >= ntiles || c >= nc) return;

    const auto rs = make_rsrc(u, state_bytes);
    const auto ro = make_rsrc(out, state_bytes);
    const auto g = geom[c];
    const T irho_c = a.inv_rho ? a.inv_rho[c] : T(1);
    const uint32_t own = tile_off<T>(c, nm);
    PnFaces<MF, T> F;
    pn_faces<MF>(g, a, c, nm, irho_c, F);
    const PnUpdate<T, typename ArgsOf<T>::type> upd(a, (T)g.inv_area, c);

    for (int k0 = 0; k0 < nm; k0 += CH) {
        T acc[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) acc[j] = T(0);
        for (int m = 0; m < nm; ++m) {
            T X, Y, P, Q;
            pn_gather<MF>(rs, F, a, own, (uint32_t)m * kPlane, m, nm, irho_c, X, Y, P, Q);
            const T* w = W + ((size_t)m * nmp + k0) * 4;
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                acc[j] = fma(X, w[4 * j + 0], acc[j]);
                acc[j] = fma(Y, w[4 * j + 1], acc[j]);
                acc[j] = fma(P, w[4 * j + 2], acc[j]);
                acc[j] = fma(Q, w[4 * j + 3], acc[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int k = k0 + j;
            if (k < nm) {
                const T uk = buf_ld<T>(rs, own, (uint32_t)k * kPlane);
                buf_st<T>(upd(uk, acc[j], sig[k], k == 0), ro, own, (uint32_t)k * kPlane);
            }
        }
    }
}

// user [ncells][nm] rows <-> tiled internal layout (to_user = 0: into the tiled layout).
template <typename T>
__global__ __launch_bounds__(256) void k_pn_layout(const int64_t* __restrict__ to_user, int32_t nc,
                                                   int32_t nm, int32_t dir, const T* __restrict__ in,
                                                   T* __restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nc) return;
    const int64_t i = to_user[k];
    const int64_t t = (int64_t)(k >> 6) * nm * kTile + (k & 63);
    for (int m = 0; m < nm; ++m) {
        if (dir == 0)
            out[t + (int64_t)m * kTile] = in[i * nm + m];
        else
            out[i * nm + m] = in[t + (int64_t)m * kTile];
    }
}

template <int MF, typename T, int N = 0>
hipError_t dispatch_fused(const snrt_mesh& m, const snrt_pn& p,
                          const typename ArgsOf<T>::type& a, const T* W, const T* sig,
                          const T* u, T* out, hipStream_t st) {
    if constexpr (N > pn::max_fused_degree<T>()) {
        return hipErrorInvalidValue;
    } else {
        if (p.degree == N) return launch_fused_t<N, MF, T>(m, p, a, W, sig, u, out, st);
        return dispatch_fused<MF, T, N + 1>(m, p, a, W, sig, u, out, st);
    }
}

template <typename T>
hipError_t launch_pn_t(const snrt_mesh& m, const snrt_pn& p, const typename ArgsOf<T>::type& a,
                       const T* W, const T* sig, const T* u, T* out, hipStream_t st) {
    if (m.nc == 0) return hipSuccess;
    if constexpr (sizeof(T) == 4) {
        if (p.degree == pn::kFusedHighDegree) return launch_pn_fused_high32(m, p, a, u, out, st);
    }
    if (p.degree <= pn::max_fused_degree<T>()) {
        return m.mf == 3 ? dispatch_fused<3, T>(m, p, a, W, sig, u, out, st)
                         : dispatch_fused<4, T>(m, p, a, W, sig, u, out, st);
    }
    const int32_t ntiles = (int32_t)((m.nc + kTile - 1) / kTile);
    const int blocks = (ntiles + 3) / 4;
    constexpr int CH = sizeof(T) == 4 ? kPnChunk32 : kPnChunk64;
    using G = typename GeomOf<T>::type;
    const G* geom;
    if constexpr (sizeof(T) == 4) geom = m.geom32; else geom = m.geom64;
    if (m.mf == 3)
        hipLaunchKernelGGL((k_pn_generic<CH, 3, T>), dim3(blocks), dim3(256), 0, st, geom,
                           (int32_t)m.nc, ntiles, p.nm, p.nmp, W, sig, a, u, out,
                           state_bytes<T>(m, p.nm));
    else
        hipLaunchKernelGGL((k_pn_generic<CH, 4, T>), dim3(blocks), dim3(256), 0, st, geom,
                           (int32_t)m.nc, ntiles, p.nm, p.nmp, W, sig, a, u, out,
                           state_bytes<T>(m, p.nm));
    return hipGetLastError();
}

}  // namespace

hipError_t launch_pn32(const snrt_mesh& m, const snrt_pn& p, const StepArgs32& a, const float* u,
                       float* out, hipStream_t st) {
    return launch_pn_t<float>(m, p, a, p.w32, p.sig32, u, out, st);
}

hipError_t launch_pn64(const snrt_mesh& m, const snrt_pn& p, const StepArgs64& a, const double* u,
                       double* out, hipStream_t st) {
    return launch_pn_t<double>(m, p, a, p.w64, p.sig64, u, out, st);
}

hipError_t launch_pn_layout(const snrt_mesh& m, int32_t nm, int to_user, int elem_bytes,
                            const void* in, void* out, hipStream_t st) {
    if (m.nc == 0) return hipSuccess;
    const int blocks = (int)((m.nc + 255) / 256);
    if (elem_bytes == 4)
        hipLaunchKernelGGL(k_pn_layout<float>, dim3(blocks), dim3(256), 0, st, m.d_to_user,
                           (int32_t)m.nc, nm, to_user, static_cast<const float*>(in),
                           static_cast<float*>(out));
    else
        hipLaunchKernelGGL(k_pn_layout<double>, dim3(blocks), dim3(256), 0, st, m.d_to_user,
                           (int32_t)m.nc, nm, to_user, static_cast<const double*>(in),
                           static_cast<double*>(out));
    return hipGetLastError();
}

}  // namespace snrt
