// Explicit S_N step and its adjoint on gfx950.
//
// One wavefront owns one cell; lane l owns the V contiguous ordinates [l*V, l*V+V) of that
// cell (psi is [cell][ordinate], ordinates fastest), so the own row and every neighbour row
// are read with fully coalesced 16-byte loads.  The cell's geometry record is wave-uniform
// and arrives through scalar loads.  Isotropic scattering is a wavefront reduction of the
// cell's own row; dense scattering reads the GEMM result S = Psi B.
//
// Forward (Sec. 4.2, eq. upwind1stOrder2; eq. SNEqns / BoltzmannCSDTrafo):
//   psi'_q = psi_q (1 - dt a_t sig_t) - dt/A sum_f s_fq u_up + dt a_s sig_s S_q + dt q_src,
//   s_fq = Omega_q . n_f, u_up = own u if s_fq > 0 else neighbour u / boundary ghost.
// Adjoint (exact transpose of the linear part; a downwind gather):
//   lam_q = l_q (1 - dt a_t sig_t) - dt/rho sum_{f: s>0} s (l_q/A - l_nbr,q/A_nbr)
//           + dt a_s sig_s (B^T-side scattering),
// plus per-cell gradient sums, one wavefront reduction each.
#include <type_traits>

#include "snrt_internal.h"

namespace snrt {

template <typename T> struct GeomOf;
template <> struct GeomOf<float> { using type = CellGeom32; };
template <> struct GeomOf<double> { using type = CellGeom64; };

template <typename T> struct ArgsOf;
template <> struct ArgsOf<float> { using type = StepArgs32; };
template <> struct ArgsOf<double> { using type = StepArgs64; };

// Load / store V contiguous elements of one lane.  EXACT: the lane's slice is in range and
// 16-byte aligned when V*sizeof(T) >= 16 (the row length is a multiple of 64 elements).
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

template <int V, bool EXACT, typename T>
__device__ __forceinline__ void load_slice(const T* __restrict__ row, int q0, int nq, T (&r)[V]) {
    if constexpr (EXACT) {
        constexpr int B = V * (int)sizeof(T);
        if constexpr (B % 16 == 0) {
            const f32x4* p = reinterpret_cast<const f32x4*>(row + q0);
#pragma unroll
            for (int i = 0; i < B / 16; ++i) {
                f32x4 v = p[i];
                __builtin_memcpy(&r[i * (16 / sizeof(T))], &v, 16);
            }
        } else if constexpr (B == 8) {
            f32x2 v = *reinterpret_cast<const f32x2*>(row + q0);
            __builtin_memcpy(&r[0], &v, 8);
        } else {
            r[0] = row[q0];
        }
    } else {
#pragma unroll
        for (int j = 0; j < V; ++j) r[j] = (q0 + j < nq) ? row[q0 + j] : T(0);
    }
}

// Output rows are written once and not re-read by this kernel: stream them past the caches.
template <int V, bool EXACT, typename T>
__device__ __forceinline__ void store_slice(T* __restrict__ row, int q0, int nq, const T (&r)[V]) {
    if constexpr (EXACT) {
        constexpr int B = V * (int)sizeof(T);
        if constexpr (B % 16 == 0) {
            f32x4* p = reinterpret_cast<f32x4*>(row + q0);
#pragma unroll
            for (int i = 0; i < B / 16; ++i) {
                f32x4 v;
                __builtin_memcpy(&v, &r[i * (16 / sizeof(T))], 16);
                __builtin_nontemporal_store(v, &p[i]);
            }
        } else if constexpr (B == 8) {
            f32x2 v;
            __builtin_memcpy(&v, &r[0], 8);
            __builtin_nontemporal_store(v, reinterpret_cast<f32x2*>(row + q0));
        } else {
            __builtin_nontemporal_store(r[0], row + q0);
        }
    } else {
#pragma unroll
        for (int j = 0; j < V; ++j)
            if (q0 + j < nq) row[q0 + j] = r[j];
    }
}

// Butterfly all-reduce over the 64 lanes; every lane ends with the same (bitwise) value.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// --------------------------------------------------------------------------- forward step

template <int V, bool EXACT, bool DENSE, typename T>
__global__ __launch_bounds__(kStepBlock) void k_step(
    const typename GeomOf<T>::type* __restrict__ geom, int64_t nc, int32_t mf, int32_t nq,
    const T* __restrict__ tab, typename ArgsOf<T>::type a, const T* __restrict__ psi_in,
    T* __restrict__ psi_out, const T* __restrict__ S)
{
    const int64_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t c = lb * kCellsPerBlock + wave;
    if (c >= nc) return;
    const int q0 = lane * V;

    T ox[V], oy[V], wi[V];
    load_slice<V, EXACT>(tab, q0, nq, ox);
    load_slice<V, EXACT>(tab + nq, q0, nq, oy);
    load_slice<V, EXACT>(tab + 3 * nq, q0, nq, wi);

    const auto* g = geom + c;
    int32_t nbr[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) nbr[f] = (f < mf) ? g->nbr[f] : kUnusedFace;

    T p[V];
    load_slice<V, EXACT>(psi_in + c * (int64_t)nq, q0, nq, p);
    T up[4][V];
    T irho_n[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        irho_n[f] = T(1);
        if (nbr[f] >= 0) {
            load_slice<V, EXACT>(psi_in + (int64_t)nbr[f] * nq, q0, nq, up[f]);
            if (a.inv_rho) irho_n[f] = a.inv_rho[nbr[f]];
        } else if (nbr[f] != kUnusedFace && !a.neumann && a.inflow) {
            load_slice<V, EXACT>(a.inflow + (int64_t)(-1 - nbr[f]) * nq, q0, nq, up[f]);
            irho_n[f] = a.inflow_scale;
        } else {
#pragma unroll
            for (int j = 0; j < V; ++j) up[f][j] = T(0);
            irho_n[f] = T(0);
        }
    }

    T src[V];
    if constexpr (DENSE) {
        load_slice<V, EXACT>(S + c * (int64_t)nq, q0, nq, src);
    } else {
        T part = T(0);
#pragma unroll
        for (int j = 0; j < V; ++j) part += wi[j] * p[j];
        const T phi = wave_sum(part);          // (1/4pi) sum_p w_p psi_p
#pragma unroll
        for (int j = 0; j < V; ++j) src[j] = phi;
    }

    const T irho = a.inv_rho ? a.inv_rho[c] : T(1);
    T u[V], acc[V];
#pragma unroll
    for (int j = 0; j < V; ++j) {
        u[j] = p[j] * irho;
        acc[j] = T(0);
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        if (nbr[f] == kUnusedFace) continue;
        const T nx = g->n[f][0], ny = g->n[f][1];
        const bool own_ghost = (nbr[f] < 0) && a.neumann;
#pragma unroll
        for (int j = 0; j < V; ++j) {
            const T s = ox[j] * nx + oy[j] * ny;
            const T ub = own_ghost ? u[j] : up[f][j] * irho_n[f];
            acc[j] += (s > T(0)) ? s * u[j] : s * ub;
        }
    }

    const T keep = T(1) - a.dt * a.alpha_t * a.sigma_t[c];
    const T cflux = a.dt * g->inv_area;
    const T cscat = a.dt * a.alpha_s * a.sigma_s[c];
    const T csrc = a.source ? a.dt * a.source[c] : T(0);
    T o[V];
#pragma unroll
    for (int j = 0; j < V; ++j) o[j] = p[j] * keep - cflux * acc[j] + cscat * src[j] + csrc;
    store_slice<V, EXACT>(psi_out + c * (int64_t)nq, q0, nq, o);
}

// --------------------------------------------------------------------------- adjoint step

template <int V, bool EXACT, bool DENSE, typename T>
__global__ __launch_bounds__(kStepBlock) void k_adjoint(
    const typename GeomOf<T>::type* __restrict__ geom, int64_t nc, int32_t mf, int32_t nq,
    const T* __restrict__ tab, typename ArgsOf<T>::type a, const T* __restrict__ psi_n,
    const T* __restrict__ lam_np1, T* __restrict__ lam_n, T* __restrict__ g_t,
    T* __restrict__ g_s, T* __restrict__ g_r, const T* __restrict__ G)
{
    const int64_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t c = lb * kCellsPerBlock + wave;
    if (c >= nc) return;
    const int q0 = lane * V;

    T ox[V], oy[V], wi[V];
    load_slice<V, EXACT>(tab, q0, nq, ox);
    load_slice<V, EXACT>(tab + nq, q0, nq, oy);
    load_slice<V, EXACT>(tab + 3 * nq, q0, nq, wi);

    const auto* g = geom + c;
    int32_t nbr[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) nbr[f] = (f < mf) ? g->nbr[f] : kUnusedFace;

    T l[V], p[V];
    load_slice<V, EXACT>(lam_np1 + c * (int64_t)nq, q0, nq, l);
    load_slice<V, EXACT>(psi_n + c * (int64_t)nq, q0, nq, p);
    T ln[4][V];
    T ia_n[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        ia_n[f] = T(0);
        if (nbr[f] >= 0) {
            load_slice<V, EXACT>(lam_np1 + (int64_t)nbr[f] * nq, q0, nq, ln[f]);
            ia_n[f] = geom[nbr[f]].inv_area;
        } else {
#pragma unroll
            for (int j = 0; j < V; ++j) ln[f][j] = T(0);
        }
    }

    const T ia = g->inv_area;
    T x[V];
#pragma unroll
    for (int j = 0; j < V; ++j) x[j] = T(0);
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        if (nbr[f] == kUnusedFace) continue;
        const T nx = g->n[f][0], ny = g->n[f][1];
        const bool interior = nbr[f] >= 0;
        const bool all_signs = !interior && a.neumann;   // Neumann ghost = own value
#pragma unroll
        for (int j = 0; j < V; ++j) {
            const T s = ox[j] * nx + oy[j] * ny;
            const T d = l[j] * ia - ln[f][j] * ia_n[f];
            x[j] += (s > T(0) || all_signs) ? s * d : T(0);
        }
    }

    const T irho = a.inv_rho ? a.inv_rho[c] : T(1);
    const T keep = T(1) - a.dt * a.alpha_t * a.sigma_t[c];
    const T cscat = a.dt * a.alpha_s * a.sigma_s[c];
    const T cstream = a.dt * irho;

    T src[V];
    T part_s;                                     // per-lane part of sum_q l_q S_q
    if constexpr (DENSE) {
        load_slice<V, EXACT>(G + c * (int64_t)nq, q0, nq, src);   // (Lambda B^T)_cq
        part_s = T(0);
#pragma unroll
        for (int j = 0; j < V; ++j) part_s += p[j] * src[j];
    } else {
        T pl = T(0), pw = T(0);
#pragma unroll
        for (int j = 0; j < V; ++j) {
            pl += l[j];
            pw += wi[j] * p[j];
        }
        const T lsum = wave_sum(pl);
        const T scell = wave_sum(pw);           // isotropic S of the cell
#pragma unroll
        for (int j = 0; j < V; ++j) src[j] = wi[j] * lsum;
        part_s = (lane == 0) ? scell * lsum : T(0);
    }

    T o[V];
    T part_t = T(0), part_r = T(0);
#pragma unroll
    for (int j = 0; j < V; ++j) {
        o[j] = l[j] * keep - cstream * x[j] + cscat * src[j];
        part_t += l[j] * p[j];
        part_r += p[j] * x[j];
    }
    store_slice<V, EXACT>(lam_n + c * (int64_t)nq, q0, nq, o);

    if (g_t) {
        const T s = wave_sum(part_t);
        if (lane == 0) g_t[c] += -a.dt * a.alpha_t * s;
    }
    if (g_s) {
        const T s = wave_sum(part_s);
        if (lane == 0) g_s[c] += a.dt * a.alpha_s * s;
    }
    if (g_r) {
        const T s = wave_sum(part_r);
        if (lane == 0) g_r[c] += a.dt * irho * irho * s;
    }
}

// --------------------------------------------------------------------------- dispatch

namespace {

template <typename T, typename F>
hipError_t dispatch_v(int32_t nq, F&& f) {
    const bool exact = (nq % kWave) == 0;
    const int v = exact ? nq / kWave : (nq + kWave - 1) / kWave;
    if (exact) {
        switch (v) {
            case 1: return f(std::integral_constant<int, 1>{}, std::true_type{});
            case 2: return f(std::integral_constant<int, 2>{}, std::true_type{});
            case 4: return f(std::integral_constant<int, 4>{}, std::true_type{});
            case 8: return f(std::integral_constant<int, 8>{}, std::true_type{});
            case 16: return f(std::integral_constant<int, 16>{}, std::true_type{});
            default: break;
        }
    }
    if (v <= 1) return f(std::integral_constant<int, 1>{}, std::false_type{});
    if (v <= 2) return f(std::integral_constant<int, 2>{}, std::false_type{});
    if (v <= 4) return f(std::integral_constant<int, 4>{}, std::false_type{});
    if (v <= 8) return f(std::integral_constant<int, 8>{}, std::false_type{});
    return f(std::integral_constant<int, 16>{}, std::false_type{});
}

inline unsigned step_blocks(int64_t nc) {
    return (unsigned)((nc + kCellsPerBlock - 1) / kCellsPerBlock);
}

template <typename T>
hipError_t launch_step_t(const typename GeomOf<T>::type* geom, const snrt_mesh& m,
                         const T* tab, int32_t nq, const typename ArgsOf<T>::type& a,
                         const T* psi_in, T* psi_out, const T* S, hipStream_t st)
{
    if (m.nc == 0) return hipSuccess;
    return dispatch_v<T>(nq, [&](auto vc, auto ex) {
        constexpr int V = decltype(vc)::value;
        constexpr bool E = decltype(ex)::value;
        if (S)
            hipLaunchKernelGGL((k_step<V, E, true, T>), dim3(step_blocks(m.nc)), dim3(kStepBlock),
                               0, st, geom, m.nc, m.mf, nq, tab, a, psi_in, psi_out, S);
        else
            hipLaunchKernelGGL((k_step<V, E, false, T>), dim3(step_blocks(m.nc)),
                               dim3(kStepBlock), 0, st, geom, m.nc, m.mf, nq, tab, a, psi_in,
                               psi_out, S);
        return hipGetLastError();
    });
}

template <typename T>
hipError_t launch_adjoint_t(const typename GeomOf<T>::type* geom, const snrt_mesh& m,
                            const T* tab, int32_t nq, const typename ArgsOf<T>::type& a,
                            const T* psi_n, const T* lam_np1, T* lam_n, T* g_t, T* g_s, T* g_r,
                            const T* G, hipStream_t st)
{
    if (m.nc == 0) return hipSuccess;
    return dispatch_v<T>(nq, [&](auto vc, auto ex) {
        constexpr int V = decltype(vc)::value;
        constexpr bool E = decltype(ex)::value;
        if (G)
            hipLaunchKernelGGL((k_adjoint<V, E, true, T>), dim3(step_blocks(m.nc)),
                               dim3(kStepBlock), 0, st, geom, m.nc, m.mf, nq, tab, a, psi_n,
                               lam_np1, lam_n, g_t, g_s, g_r, G);
        else
            hipLaunchKernelGGL((k_adjoint<V, E, false, T>), dim3(step_blocks(m.nc)),
                               dim3(kStepBlock), 0, st, geom, m.nc, m.mf, nq, tab, a, psi_n,
                               lam_np1, lam_n, g_t, g_s, g_r, G);
        return hipGetLastError();
    });
}

}  // namespace

hipError_t launch_step32(const snrt_mesh& m, const snrt_quad& q, const StepArgs32& a,
                         const float* psi_in, float* psi_out, const float* S, hipStream_t st) {
    return launch_step_t<float>(m.geom32, m, q.tab32, q.nq, a, psi_in, psi_out, S, st);
}

hipError_t launch_step64(const snrt_mesh& m, const snrt_quad& q, const StepArgs64& a,
                         const double* psi_in, double* psi_out, const double* S,
                         hipStream_t st) {
    return launch_step_t<double>(m.geom64, m, q.tab64, q.nq, a, psi_in, psi_out, S, st);
}

hipError_t launch_adjoint32(const snrt_mesh& m, const snrt_quad& q, const StepArgs32& a,
                            const float* psi_n, const float* lam_np1, float* lam_n, float* g_t,
                            float* g_s, float* g_r, const float* G, hipStream_t st) {
    return launch_adjoint_t<float>(m.geom32, m, q.tab32, q.nq, a, psi_n, lam_np1, lam_n, g_t,
                                   g_s, g_r, G, st);
}

hipError_t launch_adjoint64(const snrt_mesh& m, const snrt_quad& q, const StepArgs64& a,
                            const double* psi_n, const double* lam_np1, double* lam_n,
                            double* g_t, double* g_s, double* g_r, const double* G,
                            hipStream_t st) {
    return launch_adjoint_t<double>(m.geom64, m, q.tab64, q.nq, a, psi_n, lam_np1, lam_n, g_t,
                                    g_s, g_r, G, st);
}

}  // namespace snrt
