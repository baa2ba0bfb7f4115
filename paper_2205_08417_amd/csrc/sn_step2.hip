// Second-order scheme (Sec. 4.2, second order finite volume schemes): per stage, a limited
// Green-Gauss gradient of u = psi/rho, then the explicit Euler update whose upwind flux takes
// linear reconstructions of u on both sides of every face.  The host runs two stages and
// averages (Heun).
//
// k_grad2 (one wavefront per cell or per 256-ordinate chunk of a cell, lane = V ordinates):
//   grad u_i = 1/A_i sum_f (u_i + u_f)/2 n_if          (u_f: neighbour value or ghost value)
//   Psi_i    = min_f min(1, (u_max - u_i)/d_f) if d_f > 0, min(1, (u_min - u_i)/d_f) if
//              d_f < 0, 1 otherwise;  d_f = grad u_i . r_if,  u_max/u_min over u_i and every u_f
//   G_i      = Psi_i grad u_i, stored as two rows per cell: [cell][x|y][nq].
// k_flux2:
//   u~_i = u_i + G_i . r_if,  u~_f = u_f + G_j . r_jf (r_jf = 0 on boundary faces: the ghost is
//   not reconstructed), flux = s > 0 ? s u~_i : s u~_f, and the first-order update formula;
//   the final stage writes (psi_n + update) / 2.
// Face handling is branch-free as in the first-order kernel: interior faces read the
// neighbour row scaled by its 1/rho, Dirichlet faces the inflow row scaled by inflow_scale,
// Neumann faces the own row scaled by 1/rho, vacuum faces the own row scaled by 0; an unused
// slot is the cell itself with zero normal and zero reconstruction vectors.
#include "sn_step_kernels.h"

namespace snrt {

template <typename T> struct ReconOf;
template <> struct ReconOf<float> { using type = CellRecon32; };
template <> struct ReconOf<double> { using type = CellRecon64; };

namespace {

template <typename T>
struct FaceSource {
    const T* row;
    T scale;
};

// Far side of face f of cell c: the row to read and the factor turning it into u.
template <bool RHO, typename T>
__device__ __forceinline__ FaceSource<T> face_source(int32_t j, int64_t c, T irho, int32_t nq,
                                                     const T* __restrict__ psi,
                                                     const typename ArgsOf<T>::type& a)
{
    const bool dirichlet = a.inflow != nullptr && !a.neumann;
    if (j >= 0) return {psi + (int64_t)j * nq, RHO ? a.inv_rho[j] : T(1)};
    if (dirichlet) return {a.inflow + (-1 - (int64_t)j) * nq, (T)a.inflow_scale};
    return {psi + c * nq, a.neumann ? irho : T(0)};
}

template <int V, bool EXACT, int MF, bool RHO, typename T>
__global__ __launch_bounds__(kStepBlock) void k_grad2(
    const typename GeomOf<T>::type* __restrict__ geom,
    const typename ReconOf<T>::type* __restrict__ recon, int64_t nc, int32_t nq,
    typename ArgsOf<T>::type a, const T* __restrict__ psi, T* __restrict__ G, int32_t shift)
{
    const int64_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t item = lb * kCellsPerBlock + wave;
    if (item >= (nc << shift)) return;
    const int64_t c = item >> shift;
    const int q0 = (int)(item & ((1 << shift) - 1)) * kWave * V + lane * V;
    const auto& g = geom[c];
    const auto& rc = recon[c];

    const T irho = RHO ? a.inv_rho[c] : T(1);
    T u[V];
    load_slice<V, EXACT>(psi + c * nq, q0, nq, u);
    T gx[V], gy[V], umax[V], umin[V];
#pragma unroll
    for (int k = 0; k < V; ++k) {
        u[k] *= irho;
        gx[k] = gy[k] = T(0);
        umax[k] = umin[k] = u[k];
    }
#pragma unroll
    for (int f = 0; f < MF; ++f) {
        const FaceSource<T> fs = face_source<RHO>(g.nbr[f], c, irho, nq, psi, a);
        T uf[V];
        load_slice<V, EXACT>(fs.row, q0, nq, uf);
        const T nx = g.n[f][0], ny = g.n[f][1];
#pragma unroll
        for (int k = 0; k < V; ++k) {
            uf[k] *= fs.scale;
            const T avg = T(0.5) * (u[k] + uf[k]);
            gx[k] += avg * nx;
            gy[k] += avg * ny;
            umax[k] = uf[k] > umax[k] ? uf[k] : umax[k];
            umin[k] = uf[k] < umin[k] ? uf[k] : umin[k];
        }
    }
    T lim[V];
#pragma unroll
    for (int k = 0; k < V; ++k) {
        gx[k] *= g.inv_area;
        gy[k] *= g.inv_area;
        lim[k] = T(1);
    }
#pragma unroll
    for (int f = 0; f < MF; ++f) {
        const T rx = rc.r_own[f][0], ry = rc.r_own[f][1];
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const T d2 = gx[k] * rx + gy[k] * ry;
            T t = T(1);
            if (d2 > T(0))
                t = (umax[k] - u[k]) / d2;
            else if (d2 < T(0))
                t = (umin[k] - u[k]) / d2;
            t = t < T(1) ? t : T(1);
            lim[k] = t < lim[k] ? t : lim[k];
        }
    }
#pragma unroll
    for (int k = 0; k < V; ++k) {
        gx[k] *= lim[k];
        gy[k] *= lim[k];
    }
    store_slice<V, EXACT>(G + (2 * c) * nq, q0, nq, gx, false);
    store_slice<V, EXACT>(G + (2 * c + 1) * nq, q0, nq, gy, false);
}

template <int V, bool EXACT, int MF, bool RHO, bool DENSE, bool FINAL, typename T>
__global__ __launch_bounds__(kStepBlock) void k_flux2(
    const typename GeomOf<T>::type* __restrict__ geom,
    const typename ReconOf<T>::type* __restrict__ recon, int64_t nc, int32_t nq,
    const T* __restrict__ tab, typename ArgsOf<T>::type a, const T* __restrict__ psi,
    const T* __restrict__ G, const T* __restrict__ S, const T* __restrict__ psi_n,
    T* __restrict__ out, int32_t shift)
{
    const int64_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t item = lb * kCellsPerBlock + wave;
    if (item >= (nc << shift)) return;
    const int64_t c = item >> shift;
    const int q0 = (int)(item & ((1 << shift) - 1)) * kWave * V + lane * V;
    const auto& g = geom[c];
    const auto& rc = recon[c];

    T ox[V], oy[V], wi[V];
    load_slice<V, EXACT>(tab, q0, nq, ox);
    load_slice<V, EXACT>(tab + nq, q0, nq, oy);
    load_slice<V, EXACT>(tab + 3 * nq, q0, nq, wi);

    const T irho = RHO ? a.inv_rho[c] : T(1);
    T p[V], u[V], gxo[V], gyo[V];
    load_slice<V, EXACT>(psi + c * nq, q0, nq, p);
    load_slice<V, EXACT>(G + (2 * c) * nq, q0, nq, gxo);
    load_slice<V, EXACT>(G + (2 * c + 1) * nq, q0, nq, gyo);
#pragma unroll
    for (int k = 0; k < V; ++k) u[k] = p[k] * irho;

    T src[V];
    if constexpr (DENSE) {
        load_slice<V, EXACT>(S + c * nq, q0, nq, src);
    } else {
        T part = T(0);
#pragma unroll
        for (int k = 0; k < V; ++k) part += wi[k] * p[k];
        const T phi = cell_sum(part);           // (1/4pi) sum_p w_p psi_p
#pragma unroll
        for (int k = 0; k < V; ++k) src[k] = phi;
    }

    T acc[V];
#pragma unroll
    for (int k = 0; k < V; ++k) acc[k] = T(0);
#pragma unroll
    for (int f = 0; f < MF; ++f) {
        const int32_t j = g.nbr[f];
        const FaceSource<T> fs = face_source<RHO>(j, c, irho, nq, psi, a);
        const int64_t gj = j >= 0 ? (int64_t)j : c;     // r_far is 0 unless j is a cell
        T uf[V], gxj[V], gyj[V];
        load_slice<V, EXACT>(fs.row, q0, nq, uf);
        load_slice<V, EXACT>(G + (2 * gj) * nq, q0, nq, gxj);
        load_slice<V, EXACT>(G + (2 * gj + 1) * nq, q0, nq, gyj);
        const T nx = g.n[f][0], ny = g.n[f][1];
        const T rox = rc.r_own[f][0], roy = rc.r_own[f][1];
        const T rfx = rc.r_far[f][0], rfy = rc.r_far[f][1];
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const T s = ox[k] * nx + oy[k] * ny;
            const T ui = u[k] + gxo[k] * rox + gyo[k] * roy;
            const T uj = uf[k] * fs.scale + gxj[k] * rfx + gyj[k] * rfy;
            acc[k] += (s > T(0)) ? s * ui : s * uj;
        }
    }

    const T keep = T(1) - a.dt * a.alpha_t * a.sigma_t[c];
    const T cflux = a.dt * g.inv_area;
    const T cscat = a.dt * a.alpha_s * a.sigma_s[c];
    const T csrc = a.source ? a.dt * a.source[c] : T(0);
    T o[V];
#pragma unroll
    for (int k = 0; k < V; ++k) o[k] = p[k] * keep - cflux * acc[k] + cscat * src[k] + csrc;
    if constexpr (FINAL) {
        T pn[V];
        load_slice<V, EXACT>(psi_n + c * nq, q0, nq, pn);
#pragma unroll
        for (int k = 0; k < V; ++k) o[k] = T(0.5) * (pn[k] + o[k]);
    }
    store_slice<V, EXACT>(out + c * nq, q0, nq, o);
}

// Rows of 512 or 1024 ordinates split into 256-ordinate items when nothing couples the
// ordinates of a cell inside the kernel (the gradient always, the update with dense
// scattering); returns the chunk shift and the per-lane width through dispatch.
inline int chunk_shift(int32_t nq) { return dense_chunk_shift(nq); }

inline unsigned item_blocks(int64_t nc, int shift) {
    return (unsigned)(((nc << shift) + kCellsPerBlock - 1) / kCellsPerBlock);
}

template <typename T>
hipError_t launch_grad2_t(const snrt_mesh& m, const snrt_quad& q,
                          const typename ArgsOf<T>::type& a, const T* psi, T* G,
                          const typename GeomOf<T>::type* geom,
                          const typename ReconOf<T>::type* recon, hipStream_t st)
{
    if (m.nc == 0) return hipSuccess;
    const int shift = chunk_shift(q.nq);
    const bool rho = a.inv_rho != nullptr, mf4 = m.mf == 4;
    return dispatch_v<T>(shift ? kWave * 4 : q.nq, [&](auto vc, auto ex) {
        constexpr int V = decltype(vc)::value;
        constexpr bool E = decltype(ex)::value;
        auto go = [&](auto mfc, auto rcst) {
            constexpr int MF = decltype(mfc)::value;
            constexpr bool R = decltype(rcst)::value;
            hipLaunchKernelGGL((k_grad2<V, E, MF, R, T>), dim3(item_blocks(m.nc, shift)),
                               dim3(kStepBlock), 0, st, geom, recon, m.nc, q.nq, a, psi, G,
                               (int32_t)shift);
            return hipGetLastError();
        };
        using I3 = std::integral_constant<int, 3>;
        using I4 = std::integral_constant<int, 4>;
        if (mf4) return rho ? go(I4{}, std::true_type{}) : go(I4{}, std::false_type{});
        return rho ? go(I3{}, std::true_type{}) : go(I3{}, std::false_type{});
    });
}

template <typename T>
hipError_t launch_flux2_t(const snrt_mesh& m, const snrt_quad& q,
                          const typename ArgsOf<T>::type& a, const T* psi, const T* G,
                          const T* S, const T* psi_n, T* out, const T* tab,
                          const typename GeomOf<T>::type* geom,
                          const typename ReconOf<T>::type* recon, hipStream_t st)
{
    if (m.nc == 0) return hipSuccess;
    const bool dense = S != nullptr, fin = psi_n != nullptr;
    const int shift = dense ? chunk_shift(q.nq) : 0;
    const bool rho = a.inv_rho != nullptr, mf4 = m.mf == 4;
    return dispatch_v<T>(shift ? kWave * 4 : q.nq, [&](auto vc, auto ex) {
        constexpr int V = decltype(vc)::value;
        constexpr bool E = decltype(ex)::value;
        auto go = [&](auto mfc, auto rcst, auto dcst, auto fcst) {
            constexpr int MF = decltype(mfc)::value;
            constexpr bool R = decltype(rcst)::value;
            constexpr bool D = decltype(dcst)::value;
            constexpr bool F = decltype(fcst)::value;
            hipLaunchKernelGGL((k_flux2<V, E, MF, R, D, F, T>), dim3(item_blocks(m.nc, shift)),
                               dim3(kStepBlock), 0, st, geom, recon, m.nc, q.nq, tab, a, psi, G,
                               S, psi_n, out, (int32_t)shift);
            return hipGetLastError();
        };
        using Tt = std::true_type;
        using Ff = std::false_type;
        auto by_mf = [&](auto rcst, auto dcst, auto fcst) {
            if (mf4) return go(std::integral_constant<int, 4>{}, rcst, dcst, fcst);
            return go(std::integral_constant<int, 3>{}, rcst, dcst, fcst);
        };
        auto by_fin = [&](auto rcst, auto dcst) {
            return fin ? by_mf(rcst, dcst, Tt{}) : by_mf(rcst, dcst, Ff{});
        };
        auto by_dense = [&](auto rcst) {
            return dense ? by_fin(rcst, Tt{}) : by_fin(rcst, Ff{});
        };
        return rho ? by_dense(Tt{}) : by_dense(Ff{});
    });
}

}  // namespace

hipError_t launch_grad2_32(const snrt_mesh& m, const snrt_quad& q, const StepArgs32& a,
                           const float* psi, float* G, hipStream_t st) {
    return launch_grad2_t<float>(m, q, a, psi, G, m.geom32, m.recon32, st);
}

hipError_t launch_grad2_64(const snrt_mesh& m, const snrt_quad& q, const StepArgs64& a,
                           const double* psi, double* G, hipStream_t st) {
    return launch_grad2_t<double>(m, q, a, psi, G, m.geom64, m.recon64, st);
}

hipError_t launch_flux2_32(const snrt_mesh& m, const snrt_quad& q, const StepArgs32& a,
                           const float* psi, const float* G, const float* S,
                           const float* psi_n, float* out, hipStream_t st) {
    return launch_flux2_t<float>(m, q, a, psi, G, S, psi_n, out, q.tab32, m.geom32, m.recon32,
                                 st);
}

hipError_t launch_flux2_64(const snrt_mesh& m, const snrt_quad& q, const StepArgs64& a,
                           const double* psi, const double* G, const double* S,
                           const double* psi_n, double* out, hipStream_t st) {
    return launch_flux2_t<double>(m, q, a, psi, G, S, psi_n, out, q.tab64, m.geom64, m.recon64,
                                  st);
}

}  // namespace snrt
