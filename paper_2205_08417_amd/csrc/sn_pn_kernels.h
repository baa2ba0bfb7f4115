// P_N step on gfx950 (Sec. 3.1 P_N closure, Sec. 4.3 upwind flux with A^+ / A^-).
//
// The upwind flux of a face with outward normal n (times its length) is
//   F = sum_l n_l (A_l^{s} u_i + A_l^{-s} u_j),   s = sign(n_l),  u = moments / rho,
// and with A^{+-} = (A +- |A|)/2 this is n_l A_l (u_i + u_j)/2 + |n_l| |A_l| (u_i - u_j)/2.
// Summed over the faces of cell i the matrices factor out:
//   sum_f F = (A_x X + A_y Y + |A_x| P + |A_y| Q) / 2,
//   X = sum_f n_x,f (u_i + u_f),  Y = sum_f n_y,f (u_i + u_f),
//   P = sum_f |n_x,f| (u_i - u_f),  Q = sum_f |n_y,f| (u_i - u_f),
// so a cell gathers four vectors from its neighbours and applies four fixed operators once,
// instead of one dense product per face and direction.  A_x, A_y have at most four entries
// per row and |A_x|, |A_y| are block diagonal over the reflection classes (pn_pattern.h);
// the unrolled kernel applies exactly those entries, with the coefficients as wave-uniform
// scalar loads from a packed table.
//
// Layout: one lane per cell.  The state is stored in tiles of 64 cells, moment-major inside
// a tile: element (cell c, moment m) at ((c / 64) * nm + m) * 64 + c % 64.  A wavefront's own
// moments are 256-byte coalesced rows, a neighbour's moment is one element of a nearby
// tile, and consecutive moments of any cell are 64 elements apart, so every load of a lane
// is a 32-bit buffer offset plus a compile-time (or scalar) moment stride.
#pragma once

#include <utility>

#include "pn_pattern.h"
#include "sn_step_kernels.h"

namespace snrt {

namespace {

constexpr int kTile = 64;
constexpr double kSqrt4Pi = 3.5449077018110320546;   // int m_0 dOmega = sqrt(4 pi)

template <typename T>
__device__ __forceinline__ T buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(T) == 4) {
        const int32_t v = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
        return __builtin_bit_cast(float, v);
    } else {
        const i32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
        return __builtin_bit_cast(double, v);
    }
}

template <typename T>
__device__ __forceinline__ void buf_st(T x, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(T) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int32_t, x), r, voff, soff, 0);
    } else {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(i32x2, x), r, voff, soff, 0);
    }
}

// Byte offset of (cell x, moment 0) in the tiled layout with nm moments.
template <typename T>
__device__ __forceinline__ uint32_t tile_off(int x, int nm) {
    return ((uint32_t)(x >> 6) * (uint32_t)nm * kTile + (uint32_t)(x & 63)) * (uint32_t)sizeof(T);
}

// Per-lane face data: where the partner's moments are and how to scale them to u = mom/rho.
template <int MF, typename T>
struct PnFaces {
    uint32_t off[MF];   // partner's (tile, lane) byte offset; own cell for boundary faces
    T sc[MF];           // 1/rho of the partner (Neumann: own 1/rho; Dirichlet: 0)
    T nx[MF], ny[MF];
    int32_t ghost[MF];  // boundary face id whose ghost moments come from args.inflow, else -1
    T sx, sy, ax, ay;   // sum n_x, sum n_y, sum |n_x|, sum |n_y|
    bool any_ghost;
    // the aggregates as FMAs on the raw loads: X += cx[f] * raw_f, P += cp[f] * raw_f, ...
    T cx[MF], cy[MF], cp[MF], cq[MF];
};

template <int MF, typename T, typename G, typename A>
__device__ __forceinline__ void pn_faces(const G& g, const A& a, int c, int nm, T irho_c,
                                         PnFaces<MF, T>& F) {
    F.sx = F.sy = F.ax = F.ay = T(0);
    F.any_ghost = false;
    const uint32_t own = tile_off<T>(c, nm);
#pragma unroll
    for (int f = 0; f < MF; ++f) {
        const int32_t j = g.nbr[f];
        F.nx[f] = (T)g.n[f][0];
        F.ny[f] = (T)g.n[f][1];
        F.sx += F.nx[f];
        F.sy += F.ny[f];
        F.ax += fabs(F.nx[f]);
        F.ay += fabs(F.ny[f]);
        F.ghost[f] = -1;
        if (j >= 0) {
            F.off[f] = tile_off<T>(j, nm);
            F.sc[f] = a.inv_rho ? a.inv_rho[j] : T(1);
        } else {
            F.off[f] = own;
            F.sc[f] = a.neumann ? irho_c : T(0);
            if (!a.neumann && a.inflow) {
                F.ghost[f] = -1 - j;
                F.any_ghost = true;
            }
        }
        F.cx[f] = F.nx[f] * F.sc[f];
        F.cy[f] = F.ny[f] * F.sc[f];
        F.cp[f] = -fabs(F.nx[f]) * F.sc[f];
        F.cq[f] = -fabs(F.ny[f]) * F.sc[f];
    }
}

// The four aggregates of input moment m (soff = m * 64 * sizeof(T)).
template <int MF, typename T, typename A>
__device__ __forceinline__ void pn_gather(__amdgpu_buffer_rsrc_t rs, const PnFaces<MF, T>& F,
                                          const A& a, uint32_t own, uint32_t soff, int m, int nm,
                                          T irho_c, T& X, T& Y, T& P, T& Q) {
    const T uo = buf_ld<T>(rs, own, soff) * irho_c;
    X = F.sx * uo;
    Y = F.sy * uo;
    P = F.ax * uo;
    Q = F.ay * uo;
#pragma unroll
    for (int f = 0; f < MF; ++f) {
        T v = buf_ld<T>(rs, F.off[f], soff) * F.sc[f];
        if (F.any_ghost && F.ghost[f] >= 0)
            v += (T)a.inflow_scale * a.inflow[(int64_t)F.ghost[f] * nm + m];
        X = fma(F.nx[f], v, X);
        Y = fma(F.ny[f], v, Y);
        P = fma(-fabs(F.nx[f]), v, P);
        Q = fma(-fabs(F.ny[f]), v, Q);
    }
}

template <int KIND, typename T>
__device__ __forceinline__ T pick(T X, T Y, T P, T Q) {
    if constexpr (KIND == pn::kOpX) return X;
    else if constexpr (KIND == pn::kOpY) return Y;
    else if constexpr (KIND == pn::kOpP) return P;
    else return Q;
}

template <int N, int IDX, typename T>
__device__ __forceinline__ void apply_op(T (&acc)[pn::nmom(N)], T X, T Y, T P, T Q,
                                         const T* __restrict__ W) {
    constexpr pn::Op op = pn::OpTable<N>::ops[IDX];
    constexpr int k = op.k;
    constexpr int kind = op.kind;
    acc[k] = fma(pick<kind>(X, Y, P, Q), W[IDX], acc[k]);
}

template <int N, int S, typename T, int... I>
__device__ __forceinline__ void apply_ops(T (&acc)[pn::nmom(N)], T X, T Y, T P, T Q,
                                          const T* __restrict__ W, std::integer_sequence<int, I...>) {
    (apply_op<N, S + I>(acc, X, Y, P, Q, W), ...);
}

template <class F, int... I>
__device__ __forceinline__ void for_each_index(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}

// Cell update: u' = u + u (dt a_s s_s sigma_l(k) - dt a_t s_t) - dt/A flux_k (+ source on m_0);
// the collision factor is applied as u + u (...) so that rounding 1 + (...) to the working
// precision (an error that would repeat on every step) never scales the state.
template <typename T, typename A>
struct PnUpdate {
    T dtA, c1, c2, q0;
    __device__ __forceinline__ PnUpdate(const A& a, T inv_area, int c) {
        dtA = (T)a.dt * inv_area;
        c1 = (T)a.dt * (T)a.alpha_t * a.sigma_t[c];
        c2 = (T)a.dt * (T)a.alpha_s * a.sigma_s[c];
        q0 = a.source ? (T)a.dt * a.source[c] * (T)kSqrt4Pi : T(0);
    }
    __device__ __forceinline__ T operator()(T uk, T flux, T sig, bool first) const {
        T v = (uk + uk * (c2 * sig - c1)) - dtA * flux;
        return first ? v + q0 : v;
    }
};

// Waves per SIMD the unrolled kernel is compiled for: the accumulators of one z-parity
// subsystem plus the face data and the load pipeline (about 84 registers in FP32, 140 in
// FP64, and 24 more for a fourth face) must fit the per-wave share of the 512 VGPRs.
template <int N, int MF, typename T>
constexpr int pn_min_waves() {
    constexpr int sub = pn::SubMoments<N, 0>::count;          // the larger subsystem
    constexpr int need =
        sub * (int)(sizeof(T) / 4) + (sizeof(T) == 4 ? 84 : 140) + (MF - 3) * 24;
    constexpr int w = 512 / ((need + 7) / 8 * 8);
    return w < 1 ? 1 : w > 8 ? 8 : w;
}

// Moments whose loads are in flight ahead of the one being applied.
constexpr int kPnPrefetch = 8;
// Ghost offset of a face without an inflow ghost: past the end of the inflow buffer, so the
// buffer load returns 0 (the inflow array is below 2 GiB; checked by the library).
constexpr uint32_t kNoGhost = 0x80000000u;

// The moment loop of the unrolled kernel, a software pipeline: the loads of moment
// m + kPnPrefetch (own value and one per face) are issued before the operators of moment m
// are applied, and a scheduling barrier closes each moment so the compiler keeps that shape
// instead of hoisting every load of the unrolled loop (which exhausts the registers).  The
// own values stream from HBM, so the pipeline is deep enough to cover its latency.  GHOST:
// the wavefront holds a cell with an inflow ghost face; each face then also reads its ghost
// moments (zero for the other faces) from the inflow buffer ri.
// Own moments loaded before the cell's geometry arrives (they need no neighbour index).
constexpr int kPnEarly = 4;

// The moment loop of one z-parity subsystem (pn::SubMoments<N, PZ>), a software pipeline:
// the loads of the moment kPnPrefetch places ahead (own value and one per face) are issued
// before the operators of the current moment are applied, and a scheduling barrier closes
// each moment so the compiler keeps that shape instead of hoisting every load of the
// unrolled loop (which exhausts the registers).  GHOST: the wavefront holds a cell with an
// inflow ghost face; each face then also reads its ghost moments (zero for the other faces)
// from the inflow buffer ri.
template <bool GHOST, int N, int PZ, int MF, typename T>
__device__ __forceinline__ void pn_fused_moments(T (&acc)[pn::nmom(N)], const PnFaces<MF, T>& F,
                                                 const T (&early)[kPnEarly],
                                                 __amdgpu_buffer_rsrc_t rs,
                                                 __amdgpu_buffer_rsrc_t ri,
                                                 const uint32_t (&goff)[MF], T gscale,
                                                 uint32_t own, T irho_c, T mdt, T c1, T c2,
                                                 const T* __restrict__ W,
                                                 const T* __restrict__ sig) {
    using Sub = pn::SubMoments<N, PZ>;
    constexpr int NS = Sub::count;
    if constexpr (NS > 0) {
        // the ghost variant carries twice the loads per moment in half the depth
        constexpr int DP = GHOST ? kPnPrefetch / 2 : kPnPrefetch;
        constexpr int D = NS < DP ? NS : DP;
        constexpr int O = 1;                      // ring slot 0: the own value
        constexpr int L = O + (GHOST ? 2 * MF : MF);
        constexpr uint32_t kPlane = kTile * sizeof(T);
        auto load_faces = [&](int m, T (&raw)[L]) {
#pragma unroll
            for (int f = 0; f < MF; ++f)
                raw[O + f] = buf_ld<T>(rs, F.off[f], (uint32_t)m * kPlane);
            if constexpr (GHOST) {
#pragma unroll
                for (int f = 0; f < MF; ++f)
                    raw[O + MF + f] = buf_ld<T>(ri, goff[f], (uint32_t)m * (uint32_t)sizeof(T));
            }
        };
        // aggregate coefficients with -dt/A folded in: acc then holds -dt/A * flux directly
        const T oc[4] = {mdt * F.sx * irho_c, mdt * F.sy * irho_c, mdt * F.ax * irho_c,
                         mdt * F.ay * irho_c};
        T fc[MF][4], gc[MF][4];
#pragma unroll
        for (int f = 0; f < MF; ++f) {
            fc[f][0] = mdt * F.cx[f];
            fc[f][1] = mdt * F.cy[f];
            fc[f][2] = mdt * F.cp[f];
            fc[f][3] = mdt * F.cq[f];
            gc[f][0] = mdt * F.nx[f] * gscale;
            gc[f][1] = mdt * F.ny[f] * gscale;
            gc[f][2] = -mdt * fabs(F.nx[f]) * gscale;
            gc[f][3] = -mdt * fabs(F.ny[f]) * gscale;
        }
        T ring[D][L];
        for_each_index(
            [&](auto ic) {
                constexpr int i = decltype(ic)::value;
                constexpr int m = Sub::list[i];
                if constexpr (i < kPnEarly)
                    ring[i][0] = early[i];
                else
                    ring[i][0] = buf_ld<T>(rs, own, (uint32_t)m * kPlane);
                load_faces(m, ring[i]);
            },
            std::make_integer_sequence<int, D>{});

        for_each_index(
            [&](auto ic) {
                constexpr int i = decltype(ic)::value;
                constexpr int m = Sub::list[i];
                T raw[L];
#pragma unroll
                for (int r = 0; r < L; ++r) raw[r] = ring[i % D][r];
                if constexpr (i + D < NS) {
                    constexpr int mn = Sub::list[i + D];
                    ring[i % D][0] = buf_ld<T>(rs, own, (uint32_t)mn * kPlane);
                    load_faces(mn, ring[i % D]);
                }
                const T uo = raw[0];
                T X = oc[0] * uo, Y = oc[1] * uo, P = oc[2] * uo, Q = oc[3] * uo;
#pragma unroll
                for (int f = 0; f < MF; ++f) {
                    const T v = raw[O + f];
                    X = fma(fc[f][0], v, X);
                    Y = fma(fc[f][1], v, Y);
                    P = fma(fc[f][2], v, P);
                    Q = fma(fc[f][3], v, Q);
                    if constexpr (GHOST) {
                        const T gv = raw[O + MF + f];
                        X = fma(gc[f][0], gv, X);
                        Y = fma(gc[f][1], gv, Y);
                        P = fma(gc[f][2], gv, P);
                        Q = fma(gc[f][3], gv, Q);
                    }
                }
                // the collision term of moment m: u_m + u_m (dt a_s s_s sigma_l(m) - dt a_t s_t)
                acc[m] = fma(fma(c2, sig[m], -c1), uo, acc[m] + uo);
                constexpr int s = pn::OpTable<N>::start[m];
                constexpr int e = pn::OpTable<N>::start[m + 1];
                apply_ops<N, s>(acc, X, Y, P, Q, W, std::make_integer_sequence<int, e - s>{});
                __builtin_amdgcn_sched_barrier(0);
            },
            std::make_integer_sequence<int, NS>{});
    }
}

// One z-parity subsystem of one tile: the wavefront's lanes are the tile's cells.  acc
// accumulates u (1 - dt a_t s_t + dt a_s s_s sigma_l) - dt/A flux moment by moment, so the
// update needs no second read of the state.
template <int N, int PZ, int MF, typename T>
__device__ __forceinline__ void pn_fused_tile(const typename GeomOf<T>::type* __restrict__ geom,
                                              int c, const T* __restrict__ W,
                                              const T* __restrict__ sig,
                                              const typename ArgsOf<T>::type& a,
                                              const T* __restrict__ u, T* __restrict__ out,
                                              uint32_t state_bytes, uint32_t inflow_bytes) {
    using Sub = pn::SubMoments<N, PZ>;
    constexpr int NM = pn::nmom(N);
    constexpr int NS = Sub::count;
    constexpr uint32_t kPlane = kTile * sizeof(T);
    if constexpr (NS > 0) {
        const auto rs = make_rsrc(u, state_bytes);
        const uint32_t own = tile_off<T>(c, NM);
        T early[kPnEarly];
        for_each_index(
            [&](auto ic) {
                constexpr int i = decltype(ic)::value;
                if constexpr (i < NS)
                    early[i] = buf_ld<T>(rs, own, (uint32_t)Sub::list[i] * kPlane);
                else
                    early[i] = T(0);
            },
            std::make_integer_sequence<int, kPnEarly>{});
        const auto g = geom[c];
        const T irho_c = a.inv_rho ? a.inv_rho[c] : T(1);
        PnFaces<MF, T> F;
        pn_faces<MF>(g, a, c, NM, irho_c, F);
        const T mdt = -(T)a.dt * (T)g.inv_area;
        const T c1 = (T)a.dt * (T)a.alpha_t * a.sigma_t[c];
        const T c2 = (T)a.dt * (T)a.alpha_s * a.sigma_s[c];

        T acc[NM];
#pragma unroll
        for (int k = 0; k < NM; ++k) acc[k] = T(0);
        if (__builtin_amdgcn_ballot_w64(F.any_ghost) != 0) {
            uint32_t goff[MF];
#pragma unroll
            for (int f = 0; f < MF; ++f)
                goff[f] = F.ghost[f] >= 0 ? (uint32_t)F.ghost[f] * NM * (uint32_t)sizeof(T)
                                          : kNoGhost;
            const auto ri = make_rsrc(a.inflow, inflow_bytes);
            pn_fused_moments<true, N, PZ, MF, T>(acc, F, early, rs, ri, goff, (T)a.inflow_scale,
                                                 own, irho_c, mdt, c1, c2, W, sig);
        } else {
            const uint32_t goff[MF] = {};
            pn_fused_moments<false, N, PZ, MF, T>(acc, F, early, rs, rs, goff, T(0), own, irho_c,
                                                  mdt, c1, c2, W, sig);
        }
        if constexpr (PZ == 0) {
            // the isotropic source enters m_0 (z-even)
            if (a.source) acc[0] += (T)a.dt * a.source[c] * (T)kSqrt4Pi;
        }
        const auto ro = make_rsrc(out, state_bytes);
        for_each_index(
            [&](auto ic) {
                constexpr int m = Sub::list[decltype(ic)::value];
                buf_st<T>(acc[m], ro, own, m * kPlane);
            },
            std::make_integer_sequence<int, NS>{});
    }
}

// Fully unrolled step for degree N.  A block of 256 threads covers two tiles of 64 cells;
// its even wavefronts take a tile's z-even moments, the odd ones its z-odd moments (the
// two subsystems never meet), so each wavefront runs about half of the moment loop.  The
// packed coefficient table is read with scalar loads (uniform addresses, one per wavefront).
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// Degrees whose packed table (43 KB at degree 13) overflows the scalar cache read it from
// an LDS copy made once per block instead (measured: degree 13 0.264 -> 0.201 ms per step on
// 198 450 cells; degrees 7-9, whose tables of 6-12 KB the scalar cache holds, ran 7-9 %
// slower from LDS).
template <int N, typename T>
constexpr bool pn_table_in_lds() { return sizeof(T) == 4 && N > pn::kMaxFusedDegree; }

template <int N, int MF, typename T>
__global__ __launch_bounds__(256, (pn_min_waves<N, MF, T>())) void k_pn_fused(
    const typename GeomOf<T>::type* __restrict__ geom, int32_t nc, int32_t ntiles,
    const T* __restrict__ Wg, const T* __restrict__ sig, typename ArgsOf<T>::type a,
    const T* __restrict__ u, T* __restrict__ out, uint32_t state_bytes, uint32_t inflow_bytes) {
    const T* W = Wg;
    if constexpr (pn_table_in_lds<N, T>()) {
        constexpr int NW = pn::OpTable<N>::count;
        __shared__ __attribute__((aligned(16))) T Wl[(NW + 3) / 4 * 4];
        // 16-byte pieces, then the last NW % 4 values one by one (no read past the table)
        for (int i = (int)threadIdx.x; i < NW / 4; i += 256)
            reinterpret_cast<f32x4_t*>(Wl)[i] = reinterpret_cast<const f32x4_t*>(Wg)[i];
        if ((int)threadIdx.x < NW % 4) Wl[NW / 4 * 4 + threadIdx.x] = Wg[NW / 4 * 4 + threadIdx.x];
        __syncthreads();                  // before any wavefront of the block may leave
        W = Wl;
    }
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int tile = (int)(blk * 2 + (threadIdx.x >> 7));
    const int c = tile * kTile + (int)(threadIdx.x & 63);
    if (tile >= ntiles || c >= nc) return;
    if (((threadIdx.x >> 6) & 1) == 0)
        pn_fused_tile<N, 0, MF, T>(geom, c, W, sig, a, u, out, state_bytes, inflow_bytes);
    else
        pn_fused_tile<N, 1, MF, T>(geom, c, W, sig, a, u, out, state_bytes, inflow_bytes);
}

template <typename T>
uint32_t state_bytes(const snrt_mesh& m, int nm) {
    return (uint32_t)(((m.nc + kTile - 1) / kTile) * (int64_t)nm * kTile * (int64_t)sizeof(T));
}

template <int N, int MF, typename T>
hipError_t launch_fused_t(const snrt_mesh& m, const snrt_pn& p, const typename ArgsOf<T>::type& a,
                          const T* W, const T* sig, const T* u, T* out, hipStream_t st) {
    const int32_t ntiles = (int32_t)((m.nc + kTile - 1) / kTile);
    const int blocks = (ntiles + 1) / 2;
    using G = typename GeomOf<T>::type;
    const G* geom;
    if constexpr (sizeof(T) == 4) geom = m.geom32; else geom = m.geom64;
    const uint32_t inflow_bytes =
        a.inflow ? (uint32_t)(m.nbf * (int64_t)p.nm * (int64_t)sizeof(T)) : 0u;
    hipLaunchKernelGGL((k_pn_fused<N, MF, T>), dim3(blocks), dim3(256), 0, st, geom,
                       (int32_t)m.nc, ntiles, W, sig, a, u, out, state_bytes<T>(m, p.nm),
                       inflow_bytes);
    return hipGetLastError();
}

// ---------------------------------------------------------------- matrix-core form
//
// Inside each reflection class |A_x| and |A_y| are dense (pn_pattern.h), and their part of
// the flux, sum over the class's inputs m of |A_x|[k][m] P_m + |A_y|[k][m] Q_m into every
// output k of the class, is 85 % of the coefficient applications at degree 13.  The
// matrix-core step runs the moment loop class by class (pn::ClassOrder), keeps the sparse
// A_x X and A_y Y coefficients, the collision term and the gathers on the vector unit, and
// stages each input's P and Q in LDS (a row per cell, P in columns 0-31, Q in 32-63).  After
// a class's last input the class block D = W_c [P; Q] (W_c: 32 outputs x 64 stacked inputs,
// zero-padded) runs as 4 K steps of v_mfma_f32_32x32x16_f16 per 32-cell half, in FP16 hi+lo
// with three products (hi hi, hi lo, lo hi) as the scattering product does: each cell's
// staged values are scaled by 2^e_c (their largest magnitude into [2^13, 2^14)), the
// coefficients by a per-class 2^e_W prepared on the host, and the accumulators scaled back
// exactly.  The accumulators hold rows = outputs, columns = cells; one v_permlane32_swap per
// register pair turns the two halves into lane-per-cell rows that are added to the vector
// accumulators.
typedef _Float16 f16x8_pn __attribute__((ext_vector_type(8)));
typedef float f32x16_pn __attribute__((ext_vector_type(16)));

constexpr int kPnStageRow = 68;                      // floats per staged cell row (64 + 4)
constexpr int kPnStageWave = kTile * kPnStageRow;    // floats per wavefront

template <int N, int IDX>
__device__ __forceinline__ void apply_sparse_op(float (&acc)[pn::nmom(N)], float X, float Y,
                                                const float* __restrict__ Ws) {
    constexpr pn::Op op = pn::OpTable<N>::ops[IDX];
    constexpr int si = pn::SparseOps<N>::sidx[IDX];
    if constexpr (si >= 0) acc[op.k] = fma(op.kind == pn::kOpX ? X : Y, Ws[si], acc[op.k]);
}

template <int N, int S, int... I>
__device__ __forceinline__ void apply_sparse_ops(float (&acc)[pn::nmom(N)], float X, float Y,
                                                 const float* __restrict__ Ws,
                                                 std::integer_sequence<int, I...>) {
    (apply_sparse_op<N, S + I>(acc, X, Y, Ws), ...);
}

__device__ __forceinline__ float f32_of(uint32_t u) { return __builtin_bit_cast(float, u); }
__device__ __forceinline__ uint32_t u32_of(float f) { return __builtin_bit_cast(uint32_t, f); }

// The class block of class position Q (pn::ClassOrder<N, PZ>::order[Q]) from the staged rows
// stage (this wavefront's 64 rows), added to acc.  mx: the largest staged magnitude of the
// lane's cell (reset here).  wa: the coefficient operands [class][K step][hi, lo][lane][8]
// (FP16 bits), wae: the class exponents e_W.
template <int N, int PZ, int Q>
__device__ __forceinline__ void pn_class_block(float (&acc)[pn::nmom(N)], float& mx,
                                               const float* stage,
                                               const uint16_t* __restrict__ wa,
                                               const int32_t* __restrict__ wae, int lane) {
    using CO = pn::ClassOrder<N, PZ>;
    constexpr int lc = CO::order[Q];
    constexpr int n = CO::size[lc];
    static_assert(n <= 32, "one 32-row block per class");
    int E = 0;
    (void)__builtin_frexpf(mx, &E);
    const int e = (mx > 0.0f && mx < INFINITY) ? 14 - E : 0;
    mx = 0.0f;
    // lanes l and l + 32 of half h hold cell 32 h + l % 32
    const auto es = __builtin_amdgcn_permlane32_swap((uint32_t)e, (uint32_t)e, false, false);
    const int eh[2] = {(int)es[0], (int)es[1]};
    const int ew = wae[PZ * 4 + lc];
    const uint16_t* a = wa + (size_t)(PZ * 4 + lc) * 4 * 2 * kWave * 8;
    f32x16_pn C[2];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int r = 0; r < 16; ++r) C[h][r] = 0.0f;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const f16x8_pn ahi = *reinterpret_cast<const f16x8_pn*>(a + ((s * 2 + 0) * kWave + lane) * 8);
        const f16x8_pn alo = *reinterpret_cast<const f16x8_pn*>(a + ((s * 2 + 1) * kWave + lane) * 8);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const float* row = stage + (32 * h + (lane & 31)) * kPnStageRow + 16 * s + 8 * (lane >> 5);
            const f32x4 v0 = *reinterpret_cast<const f32x4*>(row);
            const f32x4 v1 = *reinterpret_cast<const f32x4*>(row + 4);
            f16x8_pn bhi, blo;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const float x = __builtin_ldexpf(i < 4 ? v0[i] : v1[i - 4], eh[h]);
                const _Float16 xh = (_Float16)x;
                bhi[i] = xh;
                blo[i] = (_Float16)(x - (float)xh);
            }
            C[h] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ahi, bhi, C[h], 0, 0, 0);
            C[h] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ahi, blo, C[h], 0, 0, 0);
            C[h] = __builtin_amdgcn_mfma_f32_32x32x16_f16(alo, bhi, C[h], 0, 0, 0);
        }
    }
    // accumulator r of lane l: row (r/4)*8 + (l/32)*4 + r%4, column (cell of the half) l%32
    for_each_index(
        [&](auto rc) {
            constexpr int r = decltype(rc)::value;
            constexpr int i0 = (r / 4) * 8 + (r % 4), i1 = i0 + 4;
            if constexpr (i0 < n) {
                constexpr int k0 = CO::at(lc, i0);
                constexpr int k1 = i1 < n ? CO::at(lc, i1) : 0;
                const float c0 = __builtin_ldexpf(C[0][r], -(eh[0] + ew));
                const float c1 = __builtin_ldexpf(C[1][r], -(eh[1] + ew));
                const auto sw = __builtin_amdgcn_permlane32_swap(u32_of(c0), u32_of(c1), false, false);
                acc[k0] += f32_of(sw[0]);
                if constexpr (i1 < n) acc[k1] += f32_of(sw[1]);
            }
        },
        std::make_integer_sequence<int, 16>{});
}

// The moment loop of one z-parity subsystem in class order, with the load pipeline of
// pn_fused_moments; the class blocks run after each class's last input.
template <bool GHOST, int N, int PZ, int MF>
__device__ __forceinline__ void pn_mfma_moments(float (&acc)[pn::nmom(N)],
                                                const PnFaces<MF, float>& F,
                                                __amdgpu_buffer_rsrc_t rs,
                                                __amdgpu_buffer_rsrc_t ri,
                                                const uint32_t (&goff)[MF], float gscale,
                                                uint32_t own, float irho_c, float mdt, float c1,
                                                float c2, const float* __restrict__ Ws,
                                                const float* __restrict__ sig, float* stage,
                                                const uint16_t* __restrict__ wa,
                                                const int32_t* __restrict__ wae, int lane) {
    using T = float;
    using CO = pn::ClassOrder<N, PZ>;
    constexpr int NS = CO::count;
    constexpr int D = NS < kPnPrefetch ? NS : (GHOST ? kPnPrefetch / 2 : kPnPrefetch);
    constexpr int O = 1;
    constexpr int L = O + (GHOST ? 2 * MF : MF);
    constexpr uint32_t kPlane = kTile * sizeof(T);
    auto load_faces = [&](int m, T (&raw)[L]) {
#pragma unroll
        for (int f = 0; f < MF; ++f) raw[O + f] = buf_ld<T>(rs, F.off[f], (uint32_t)m * kPlane);
        if constexpr (GHOST) {
#pragma unroll
            for (int f = 0; f < MF; ++f)
                raw[O + MF + f] = buf_ld<T>(ri, goff[f], (uint32_t)m * (uint32_t)sizeof(T));
        }
    };
    const T oc[4] = {mdt * F.sx * irho_c, mdt * F.sy * irho_c, mdt * F.ax * irho_c,
                     mdt * F.ay * irho_c};
    T fc[MF][4], gc[MF][4];
#pragma unroll
    for (int f = 0; f < MF; ++f) {
        fc[f][0] = mdt * F.cx[f];
        fc[f][1] = mdt * F.cy[f];
        fc[f][2] = mdt * F.cp[f];
        fc[f][3] = mdt * F.cq[f];
        gc[f][0] = mdt * F.nx[f] * gscale;
        gc[f][1] = mdt * F.ny[f] * gscale;
        gc[f][2] = -mdt * fabs(F.nx[f]) * gscale;
        gc[f][3] = -mdt * fabs(F.ny[f]) * gscale;
    }
    float* srow = stage + lane * kPnStageRow;
    T mx = T(0);
    T ring[D][L];
    for_each_index(
        [&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int m = CO::list[i];
            ring[i][0] = buf_ld<T>(rs, own, (uint32_t)m * kPlane);
            load_faces(m, ring[i]);
        },
        std::make_integer_sequence<int, D>{});

    for_each_index(
        [&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int m = CO::list[i];
            T raw[L];
#pragma unroll
            for (int r = 0; r < L; ++r) raw[r] = ring[i % D][r];
            if constexpr (i + D < NS) {
                constexpr int mn = CO::list[i + D];
                ring[i % D][0] = buf_ld<T>(rs, own, (uint32_t)mn * kPlane);
                load_faces(mn, ring[i % D]);
            }
            const T uo = raw[0];
            T X = oc[0] * uo, Y = oc[1] * uo, P = oc[2] * uo, Q = oc[3] * uo;
#pragma unroll
            for (int f = 0; f < MF; ++f) {
                const T v = raw[O + f];
                X = fma(fc[f][0], v, X);
                Y = fma(fc[f][1], v, Y);
                P = fma(fc[f][2], v, P);
                Q = fma(fc[f][3], v, Q);
                if constexpr (GHOST) {
                    const T gv = raw[O + MF + f];
                    X = fma(gc[f][0], gv, X);
                    Y = fma(gc[f][1], gv, Y);
                    P = fma(gc[f][2], gv, P);
                    Q = fma(gc[f][3], gv, Q);
                }
            }
            acc[m] = fma(fma(c2, sig[m], -c1), uo, acc[m] + uo);
            constexpr int s = pn::OpTable<N>::start[m];
            constexpr int e = pn::OpTable<N>::start[m + 1];
            apply_sparse_ops<N, s>(acc, X, Y, Ws, std::make_integer_sequence<int, e - s>{});
            // stage P and Q of this input in its class column
            constexpr int t = CO::local[m];
            srow[t] = P;
            srow[32 + t] = Q;
            mx = fmaxf(mx, fmaxf(fabsf(P), fabsf(Q)));
            __builtin_amdgcn_sched_barrier(0);
            // after the last input of class position q: its class block
            constexpr int q = (i < CO::size[CO::order[0]]) ? 0
                              : (i < CO::size[CO::order[0]] + CO::size[CO::order[1]]) ? 1
                              : (i < CO::size[CO::order[0]] + CO::size[CO::order[1]] +
                                         CO::size[CO::order[2]]) ? 2 : 3;
            constexpr int endq = CO::size[CO::order[0]] + (q >= 1 ? CO::size[CO::order[1]] : 0) +
                                 (q >= 2 ? CO::size[CO::order[2]] : 0) +
                                 (q >= 3 ? CO::size[CO::order[3]] : 0);
            if constexpr (i + 1 == endq) {
                pn_class_block<N, PZ, q>(acc, mx, stage, wa, wae, lane);
                // a smaller next class leaves this class's values in its padding columns:
                // clear them (the class blocks read all 32 columns of P and of Q)
                if constexpr (q < 3) {
                    constexpr int nn = CO::size[CO::order[q + 1]], nc = CO::size[CO::order[q]];
#pragma unroll
                    for (int z = nn; z < nc; ++z) {
                        srow[z] = 0.0f;
                        srow[32 + z] = 0.0f;
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        },
        std::make_integer_sequence<int, NS>{});
}

template <int N, int PZ, int MF>
__device__ __forceinline__ void pn_mfma_tile(const CellGeom32* __restrict__ geom, int c, bool live,
                                             const float* __restrict__ Ws,
                                             const float* __restrict__ sig, const StepArgs32& a,
                                             const float* __restrict__ u, float* __restrict__ out,
                                             uint32_t state_bytes, uint32_t inflow_bytes,
                                             float* stage, const uint16_t* __restrict__ wa,
                                             const int32_t* __restrict__ wae, int lane) {
    using T = float;
    using CO = pn::ClassOrder<N, PZ>;
    constexpr int NM = pn::nmom(N);
    constexpr uint32_t kPlane = kTile * sizeof(T);
    const auto rs = make_rsrc(u, state_bytes);
    const uint32_t own = tile_off<T>(c, NM);
    const auto g = geom[c];
    const T irho_c = a.inv_rho ? a.inv_rho[c] : T(1);
    PnFaces<MF, T> F;
    pn_faces<MF>(g, a, c, NM, irho_c, F);
    const T mdt = -a.dt * g.inv_area;
    const T c1 = a.dt * a.alpha_t * a.sigma_t[c];
    const T c2 = a.dt * a.alpha_s * a.sigma_s[c];
    T acc[NM];
#pragma unroll
    for (int k = 0; k < NM; ++k) acc[k] = T(0);
    if (__builtin_amdgcn_ballot_w64(F.any_ghost) != 0) {
        uint32_t goff[MF];
#pragma unroll
        for (int f = 0; f < MF; ++f)
            goff[f] = F.ghost[f] >= 0 ? (uint32_t)F.ghost[f] * NM * (uint32_t)sizeof(T) : kNoGhost;
        const auto ri = make_rsrc(a.inflow, inflow_bytes);
        pn_mfma_moments<true, N, PZ, MF>(acc, F, rs, ri, goff, a.inflow_scale, own,
                                         irho_c, mdt, c1, c2, Ws, sig, stage, wa, wae, lane);
    } else {
        const uint32_t goff[MF] = {};
        pn_mfma_moments<false, N, PZ, MF>(acc, F, rs, rs, goff, 0.0f, own, irho_c, mdt,
                                          c1, c2, Ws, sig, stage, wa, wae, lane);
    }
    if constexpr (PZ == 0) {
        if (a.source) acc[0] += a.dt * a.source[c] * (T)kSqrt4Pi;
    }
    if (!live) return;
    const auto ro = make_rsrc(out, state_bytes);
    for_each_index(
        [&](auto ic) {
            constexpr int m = CO::list[decltype(ic)::value];
            buf_st<T>(acc[m], ro, own, m * kPlane);
        },
        std::make_integer_sequence<int, CO::count>{});
}

// Matrix-core step of degree N (FP32 state): two tiles per block, even wavefronts the z-even
// subsystem, odd ones the z-odd.  Every lane of a wavefront takes part in the matrix products
// (their operands span the wavefront), so lanes past the last cell run a copy of the last
// cell and only skip the stores.
template <int N, int MF>
__global__ __launch_bounds__(256, 2) void k_pn_mfma(const CellGeom32* __restrict__ geom,
                                                    int32_t nc, int32_t ntiles,
                                                    const float* __restrict__ Ws,
                                                    const float* __restrict__ sig, StepArgs32 a,
                                                    const float* __restrict__ u,
                                                    float* __restrict__ out, uint32_t state_bytes,
                                                    uint32_t inflow_bytes,
                                                    const uint16_t* __restrict__ wa,
                                                    const int32_t* __restrict__ wae) {
    __shared__ __attribute__((aligned(16))) float stage_all[4 * kPnStageWave];
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int tile = (int)(blk * 2 + (threadIdx.x >> 7));
    if (tile >= ntiles) return;
    const int wave = (int)(threadIdx.x >> 6);
    const int lane = (int)(threadIdx.x & 63);
    float* stage = stage_all + wave * kPnStageWave;
    float* srow = stage + lane * kPnStageRow;
#pragma unroll
    for (int i = 0; i < kPnStageRow; i += 4)
        *reinterpret_cast<f32x4*>(srow + i) = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const int cl = tile * kTile + lane;
    const bool live = cl < nc;
    const int c = live ? cl : nc - 1;
    if ((wave & 1) == 0)
        pn_mfma_tile<N, 0, MF>(geom, c, live, Ws, sig, a, u, out, state_bytes, inflow_bytes,
                               stage, wa, wae, lane);
    else
        pn_mfma_tile<N, 1, MF>(geom, c, live, Ws, sig, a, u, out, state_bytes, inflow_bytes,
                               stage, wa, wae, lane);
}

template <int N, int MF>
hipError_t launch_mfma_t(const snrt_mesh& m, const snrt_pn& p, const StepArgs32& a,
                         const float* u, float* out, hipStream_t st) {
    const int32_t ntiles = (int32_t)((m.nc + kTile - 1) / kTile);
    const int blocks = (ntiles + 1) / 2;
    const uint32_t inflow_bytes =
        a.inflow ? (uint32_t)(m.nbf * (int64_t)p.nm * (int64_t)sizeof(float)) : 0u;
    hipLaunchKernelGGL((k_pn_mfma<N, MF>), dim3(blocks), dim3(256), 0, st, m.geom32,
                       (int32_t)m.nc, ntiles, p.wsp32, p.sig32, a, u, out,
                       state_bytes<float>(m, p.nm), inflow_bytes, p.wa16, p.wae);
    return hipGetLastError();
}

}  // namespace

}  // namespace snrt
