// Explicit S_N step and its adjoint on gfx950 (kernel templates; instantiated by
// sn_step_f32.hip, sn_step_f64.hip and sn_adjoint.hip).
//
// One wavefront owns one cell; lane l owns the V contiguous ordinates [l*V, l*V+V) of that
// cell (psi is [cell][ordinate], ordinates fastest), so the own row and every neighbour row
// are read with fully coalesced 16-byte loads.  The cell's geometry record is wave-uniform
// and arrives through scalar loads.  Isotropic scattering is a wavefront reduction of the
// cell's own row; dense scattering reads the GEMM result S = Psi B.
//
// Forward (Sec. 4.2, eq. upwind1stOrder2; eq. SNEqns / BoltzmannCSDTrafo):
//   psi'_q = psi_q - dt a_t sig_t psi_q - dt/A sum_f s_fq u_up + dt a_s sig_s S_q + dt q_src,
//   s_fq = Omega_q . n_f, u_up = own u if s_fq > 0 else neighbour u / boundary ghost.
// Adjoint (exact transpose of the linear part; a downwind gather):
//   lam_q = l_q - dt a_t sig_t l_q - dt/rho sum_{f: s>0} s (l_q/A - l_nbr,q/A_nbr)
//           + dt a_s sig_s (B^T-side scattering),
// plus per-cell gradient sums, one wavefront reduction each.
//
// The absorption is applied as psi - (dt a_t sig_t) psi, never as psi (1 - dt a_t sig_t): the
// factor 1 - dt a_t sig_t rounded to the working precision carries an absolute error of up
// to half an ulp of 1 that would repeat identically on every step and compound over a long
// run (about nsteps * 3e-8 relative in FP32), while the small coefficient itself keeps full
// relative precision.  Implicit collisions divide by 1 + c the same way, as r - r c/(1 + c).
#pragma once

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
__device__ __forceinline__ void store_slice(T* __restrict__ row, int q0, int nq, const T (&r)[V],
                                            bool nt = true) {
    if constexpr (EXACT) {
        constexpr int B = V * (int)sizeof(T);
        if constexpr (B % 16 == 0) {
            f32x4* p = reinterpret_cast<f32x4*>(row + q0);
#pragma unroll
            for (int i = 0; i < B / 16; ++i) {
                f32x4 v;
                __builtin_memcpy(&v, &r[i * (16 / sizeof(T))], 16);
                if (nt)
                    __builtin_nontemporal_store(v, &p[i]);
                else
                    p[i] = v;
            }
        } else if constexpr (B == 8) {
            f32x2 v;
            __builtin_memcpy(&v, &r[0], 8);
            if (nt)
                __builtin_nontemporal_store(v, reinterpret_cast<f32x2*>(row + q0));
            else
                *reinterpret_cast<f32x2*>(row + q0) = v;
        } else {
            if (nt)
                __builtin_nontemporal_store(r[0], row + q0);
            else
                row[q0] = r[0];
        }
    } else {
#pragma unroll
        for (int j = 0; j < V; ++j)
            if (q0 + j < nq) row[q0 + j] = r[j];
    }
}

// ---------------------------------------------------------------- buffer-resource access
// Rows are addressed as 32-bit byte offsets into a buffer resource (base, size): the row
// offset is one scalar multiply, the lane offset a constant, and reads outside the buffer
// return 0 instead of faulting.  Every array the step touches is below 4 GiB (checked by
// the library before launch).

typedef int32_t i32x2 __attribute__((ext_vector_type(2)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

constexpr int32_t kRsrcWord3 = 0x00020000;   // raw buffer, 32-bit data format (CDNA)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int32_t)bytes, kRsrcWord3);
}

// V contiguous elements of this lane from the row at byte offset soff (EXACT: the row has
// 64*V elements; otherwise lanes past nq read 0).
// Cache-policy bits of buffer accesses on CDNA3/4: 1 = sc0, 2 = nt (streaming), 16 = sc1.
constexpr int kAuxDefault = 0;
constexpr int kAuxStream = 2;

template <int V, bool EXACT, typename T, int AUX = kAuxDefault>
__device__ __forceinline__ void buf_load_row(__amdgpu_buffer_rsrc_t r, uint32_t soff, int q0,
                                             int nq, T (&out)[V]) {
    if constexpr (EXACT) {
        constexpr int B = V * (int)sizeof(T);
        const uint32_t voff = (uint32_t)q0 * sizeof(T);
        if constexpr (B % 16 == 0) {
#pragma unroll
            for (int i = 0; i < B / 16; ++i) {
                i32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, voff + 16 * i, soff, AUX);
                __builtin_memcpy(&out[i * (16 / sizeof(T))], &v, 16);
            }
        } else if constexpr (B == 8) {
            i32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, AUX);
            __builtin_memcpy(&out[0], &v, 8);
        } else {
            int32_t v = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, AUX);
            __builtin_memcpy(&out[0], &v, 4);
        }
    } else {
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const int q = q0 + k < nq ? q0 + k : nq - 1;           // clamp, then zero
            T v;
            if constexpr (sizeof(T) == 4) {
                int32_t b = __builtin_amdgcn_raw_buffer_load_b32(r, (uint32_t)q * 4u, soff, AUX);
                __builtin_memcpy(&v, &b, 4);
            } else {
                i32x2 b = __builtin_amdgcn_raw_buffer_load_b64(r, (uint32_t)q * 8u, soff, AUX);
                __builtin_memcpy(&v, &b, 8);
            }
            out[k] = q0 + k < nq ? v : T(0);
        }
    }
}

template <int V, bool EXACT, typename T, int AUX = kAuxDefault>
__device__ __forceinline__ void buf_store_row(__amdgpu_buffer_rsrc_t r, uint32_t soff, int q0,
                                              int nq, const T (&in)[V]) {
    if constexpr (EXACT) {
        constexpr int B = V * (int)sizeof(T);
        const uint32_t voff = (uint32_t)q0 * sizeof(T);
        if constexpr (B % 16 == 0) {
#pragma unroll
            for (int i = 0; i < B / 16; ++i) {
                i32x4 v;
                __builtin_memcpy(&v, &in[i * (16 / sizeof(T))], 16);
                __builtin_amdgcn_raw_buffer_store_b128(v, r, voff + 16 * i, soff, AUX);
            }
        } else if constexpr (B == 8) {
            i32x2 v;
            __builtin_memcpy(&v, &in[0], 8);
            __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, soff, AUX);
        } else {
            int32_t v;
            __builtin_memcpy(&v, &in[0], 4);
            __builtin_amdgcn_raw_buffer_store_b32(v, r, voff, soff, AUX);
        }
    } else {
#pragma unroll
        for (int k = 0; k < V; ++k) {
            if (q0 + k >= nq) continue;
            if constexpr (sizeof(T) == 4) {
                int32_t b;
                __builtin_memcpy(&b, &in[k], 4);
                __builtin_amdgcn_raw_buffer_store_b32(b, r, (uint32_t)(q0 + k) * 4u, soff, AUX);
            } else {
                i32x2 b;
                __builtin_memcpy(&b, &in[k], 8);
                __builtin_amdgcn_raw_buffer_store_b64(b, r, (uint32_t)(q0 + k) * 8u, soff, AUX);
            }
        }
    }
}

// Element i of a per-cell array through a scalar load with a 32-bit byte offset.
template <typename T>
__device__ __forceinline__ T cell_val(const T* __restrict__ a, int32_t i) {
    const uint32_t off = (uint32_t)i * (uint32_t)sizeof(T);
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(a) + off);
}

template <typename G>
__device__ __forceinline__ const G* cell_rec(const G* __restrict__ g, int32_t i) {
    const uint32_t off = (uint32_t)i * (uint32_t)sizeof(G);
    return reinterpret_cast<const G*>(reinterpret_cast<const char*>(g) + off);
}

// Butterfly all-reduce over the 64 lanes; every lane ends with the same (bitwise) value.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// FP32 all-reduce without LDS traffic: DPP swaps inside each 16-lane row (xor 1, xor 2,
// half-row mirror, row mirror leave every lane of a row with the same row sum), then the
// four row sums are read into scalars and added in a fixed order.  Deterministic and
// wave-uniform.
template <int CTRL>
__device__ __forceinline__ float dpp_partner(float v) {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ float wave_sum_dpp(float v) {
    v += dpp_partner<0xB1>(v);    // quad_perm(1,0,3,2): lane ^ 1
    v += dpp_partner<0x4E>(v);    // quad_perm(2,3,0,1): lane ^ 2
    v += dpp_partner<0x141>(v);   // row_half_mirror: lane i <-> 7 - i within 8
    v += dpp_partner<0x140>(v);   // row_mirror: lane i <-> 15 - i within 16
    const float r0 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 0));
    const float r1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 16));
    const float r2 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 32));
    const float r3 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 48));
    return (r0 + r1) + (r2 + r3);
}

template <typename T>
__device__ __forceinline__ T cell_sum(T v) {
    if constexpr (sizeof(T) == 4)
        return wave_sum_dpp(v);
    else
        return wave_sum(v);
}

// --------------------------------------------------------------------------- forward step
//
// Persistent, XCD-partitioned launch: the grid is a multiple of the XCD count; XCD x owns
// the contiguous (Hilbert-ordered) cell range [x*cpx, (x+1)*cpx) and its waves sweep that
// range together, one cell per wave per iteration, so neighbour rows are read from the
// XCD's own L2 shortly after (or before) their owner reads them.  The ordinate table is
// loaded once per wave.  Rows are read with the default (L2-allocating) policy because each
// is read again as a neighbour; output rows are written with the streaming policy.
//
// Three-stage software pipeline with straight-line memory operations:
//   stage A (two cells ahead):  the 16-byte neighbour list (scalar load);
//   stage B (one cell ahead):   own row, the MF face rows, normals and coefficients;
//   stage C (this cell):        arithmetic and the row store.
// Every face gets a row pointer and a scale chosen with scalar selects: interior faces read
// the neighbour row scaled by its 1/rho, Dirichlet faces the inflow row scaled by
// inflow_scale, Neumann faces the cell's own row scaled by its 1/rho, vacuum and unused
// faces the cell's own row scaled by 0.  No load sits under a branch, so the waits of
// stage C cover only this cell's loads.

// Wave-uniform cell index in a scalar register (cell counts are below 2^31).
__device__ __forceinline__ int32_t uniform_cell(int32_t c) {
    return __builtin_amdgcn_readfirstlane(c);
}

template <typename T>
__device__ __forceinline__ T fma_t(T a, T b, T c) {
    if constexpr (sizeof(T) == 4)
        return __builtin_fmaf(a, b, c);
    else
        return __builtin_fma(a, b, c);
}

template <int MF>
struct NbrList {
    int32_t j[MF];
};

template <int V, int MF, bool DENSE, typename T>
struct FwdStage {
    T p[V];
    T up[MF][V];
    T src[V];
    T ghost[MF];
    T nx[MF], ny[MF];
    T irho, cabs, cflux, cscat, srcv;   // cabs = dt alpha_t sigma_t; srcv: the cell's source
};

// Buffer resources and scalars of one launch.
template <typename T>
struct FwdCtx {
    __amdgpu_buffer_rsrc_t psi, inflow, out, S;
    uint32_t row_bytes;
    const T *src_arr;
    T src_mul, inflow_scale;
    bool dirichlet, neumann;
    double* dpart;    // FP64 sum_q w_q psi_q of each work item (the fused dose), or unused
};

template <int MF, typename T>
__device__ __forceinline__ void fwd_load_nbr(NbrList<MF>& nb,
                                             const typename GeomOf<T>::type* __restrict__ geom,
                                             int32_t c)
{
    const auto* g = cell_rec(geom, c);
#pragma unroll
    for (int f = 0; f < MF; ++f) nb.j[f] = g->nbr[f];
}

// LOAD_S: read the scattering source row of a dense step from x.S (a caller that holds the
// source elsewhere fills d.src itself).
template <int V, bool EXACT, int MF, bool RHO, bool DENSE, typename T, int LA_OWN = kAuxDefault,
          int LA_NBR = kAuxDefault, bool LOAD_S = DENSE>
__device__ __forceinline__ void fwd_load_stage(FwdStage<V, MF, DENSE, T>& d, const NbrList<MF>& nb,
                                               const typename GeomOf<T>::type* __restrict__ geom,
                                               int32_t c, uint32_t cb, int32_t nq, int q0,
                                               const typename ArgsOf<T>::type& a,
                                               const FwdCtx<T>& x)
{
    const auto* g = cell_rec(geom, c);
    const uint32_t own = (uint32_t)c * x.row_bytes + cb;
    buf_load_row<V, EXACT, T, LA_OWN>(x.psi, own, q0, nq, d.p);
    d.irho = RHO ? cell_val(a.inv_rho, c) : T(1);
    // boundary faces: Dirichlet reads the inflow row (scale inflow_scale), Neumann the
    // cell's own row (scale 1/rho), vacuum the own row with scale 0
    const T bscale = x.dirichlet ? x.inflow_scale : (x.neumann ? d.irho : T(0));
#pragma unroll
    for (int f = 0; f < MF; ++f) {
        const int32_t j = nb.j[f];
        const bool bnd = j < 0;
        const int32_t bidx = x.dirichlet ? -1 - j : c;
        const uint32_t off = (uint32_t)(bnd ? bidx : j) * x.row_bytes + cb;
        const T rho_j = RHO ? cell_val(a.inv_rho, bnd ? c : j) : T(1);
        d.ghost[f] = bnd ? bscale : rho_j;
        buf_load_row<V, EXACT, T, LA_NBR>(bnd && x.dirichlet ? x.inflow : x.psi, off, q0, nq,
                                          d.up[f]);
        d.nx[f] = g->n[f][0];
        d.ny[f] = g->n[f][1];
    }
    if constexpr (DENSE && LOAD_S) buf_load_row<V, EXACT, T, kAuxStream>(x.S, own, q0, nq, d.src);
    const T st_c = cell_val(a.sigma_t, c);
    d.cabs = a.dt * a.alpha_t * st_c;
    d.cflux = a.dt * g->inv_area;
    d.cscat = a.dt * a.alpha_s * cell_val(a.sigma_s, c);
    d.srcv = cell_val(x.src_arr, c);
}

template <int V, bool EXACT, int MF, bool RHO, bool DENSE, typename T, int SA = kAuxStream,
          bool IMEX = false, bool DOSE = false>
__device__ __forceinline__ void fwd_compute(const FwdStage<V, MF, DENSE, T>& d, const T (&ox)[V],
                                            const T (&oy)[V], const T (&wi)[V], int32_t c,
                                            uint32_t cb, int32_t nq, int q0, const FwdCtx<T>& x,
                                            T w4 = T(0), const double* wd = nullptr,
                                            int32_t item = 0)
{
    if constexpr (DOSE) {
        // the dose of the state entering the step: FP64 weighted sum of this item's slice
        double sd = 0.0;
#pragma unroll
        for (int k = 0; k < V; ++k) sd += wd[k] * (double)d.p[k];
        sd = wave_sum(sd);
        if (q0 == 0) x.dpart[item] = sd;
    }
    if constexpr (IMEX) {
        // (a - c K~) psi' = b, K~ = w/(4 pi) (isotropic): with B = sum_q (w_q/4pi) b_q and
        // W = sum_q w_q/(4 pi), the scalar flux of psi' is B / (a - c W) times 4 pi, so
        // psi'_q = (b_q + c B / (a - c W)) / a  (Sherman-Morrison on the rank-one kernel),
        // a = 1 + cabs; the final division is taken as r - r y, y = cabs / (1 + cabs)
        T u[V], acc[V];
#pragma unroll
        for (int k = 0; k < V; ++k) {
            u[k] = RHO ? d.p[k] * d.irho : d.p[k];
            acc[k] = T(0);
        }
#pragma unroll
        for (int f = 0; f < MF; ++f) {
#pragma unroll
            for (int k = 0; k < V; ++k) {
                const T s = ox[k] * d.nx[f] + oy[k] * d.ny[f];
                const T ub = d.up[f][k] * d.ghost[f];
                acc[k] += (s > T(0)) ? s * u[k] : s * ub;
            }
        }
        T b[V];
        T part = T(0);
#pragma unroll
        for (int k = 0; k < V; ++k) {
            b[k] = d.p[k] - d.cflux * acc[k] + x.src_mul * d.srcv;
            part += wi[k] * b[k];
        }
        const T B = cell_sum(part);
        const T phi4 = B / (T(1) + (d.cabs - d.cscat * w4));
        const T y = d.cabs / (T(1) + d.cabs);
        T o[V];
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const T r = b[k] + d.cscat * phi4;
            o[k] = r - r * y;
        }
        buf_store_row<V, EXACT, T, SA>(x.out, (uint32_t)c * x.row_bytes + cb, q0, nq, o);
        return;
    }
    T src[V];
    if constexpr (DENSE) {
#pragma unroll
        for (int k = 0; k < V; ++k) src[k] = d.src[k];
    } else {
        T part = T(0);
#pragma unroll
        for (int k = 0; k < V; ++k) part += wi[k] * d.p[k];
        const T phi = cell_sum(part);              // (1/4pi) sum_p w_p psi_p
#pragma unroll
        for (int k = 0; k < V; ++k) src[k] = phi;
    }
    T u[V], acc[V];
#pragma unroll
    for (int k = 0; k < V; ++k) {
        u[k] = RHO ? d.p[k] * d.irho : d.p[k];
        acc[k] = T(0);
    }
    T o[V];
    if constexpr (DENSE) {
        // Dense scattering: every rounding step spelled out as an explicit FMA.  The compiler
        // contracts a product into a sum only when both sit in one basic block, which depends
        // on the caller's loop structure; written out, the step kernel and the product tiles
        // of the one-launch dense step (which inline this update in different loops) compute
        // the same bits.  The forms are the ones the compiler picks for the step kernel.
#pragma unroll
        for (int f = 0; f < MF; ++f) {
#pragma unroll
            for (int k = 0; k < V; ++k) {
                const T s = fma_t(d.nx[f], ox[k], d.ny[f] * oy[k]);
                acc[k] = fma_t(s, s > T(0) ? u[k] : d.up[f][k] * d.ghost[f], acc[k]);
            }
        }
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const T v = fma_t(-d.cflux, acc[k], fma_t(-d.p[k], d.cabs, d.p[k]));
            o[k] = fma_t(x.src_mul, d.srcv, fma_t(d.cscat, src[k], v));
        }
    } else {
#pragma unroll
        for (int f = 0; f < MF; ++f) {
#pragma unroll
            for (int k = 0; k < V; ++k) {
                const T s = ox[k] * d.nx[f] + oy[k] * d.ny[f];
                const T ub = d.up[f][k] * d.ghost[f];
                acc[k] += (s > T(0)) ? s * u[k] : s * ub;
            }
        }
#pragma unroll
        for (int k = 0; k < V; ++k)
            o[k] = (d.p[k] - d.cabs * d.p[k]) - d.cflux * acc[k] + d.cscat * src[k] +
                   x.src_mul * d.srcv;
    }
    buf_store_row<V, EXACT, T, SA>(x.out, (uint32_t)c * x.row_bytes + cb, q0, nq, o);
}

template <int V, bool EXACT, int MF, bool RHO, bool DENSE, typename T, bool IMEX, bool DOSE>
__device__ __forceinline__ void step_sweep(
    const typename GeomOf<T>::type* __restrict__ geom, int64_t nc, int32_t nq,
    const T* __restrict__ tab, const typename ArgsOf<T>::type& a, const T* __restrict__ psi_in,
    T* __restrict__ psi_out, const T* __restrict__ S, int64_t items_per_xcd, uint32_t nbf,
    int32_t shift, const double* __restrict__ wq, double* __restrict__ dpart)
{
    // Work items: with dense scattering no ordinate couples to another inside the step, so
    // a row may be cut into 2^shift chunks of 64*V ordinates, one item each (item i is chunk
    // i & (2^shift - 1) of cell i >> shift).  Isotropic scattering needs the whole row in
    // one wave (shift = 0).
    // XCD x owns items [x*ipx, (x+1)*ipx) and all its waves sweep that range together,
    // four consecutive items per block per iteration: a row is read as a neighbour within a
    // short window of its owner's read, while it is still in the XCD's L2.  ipx and the
    // sweep stride are multiples of 4 >= 2^shift, so a wave keeps one chunk throughout.
    const int x = blockIdx.x % kNumXcd;
    const int kx = blockIdx.x / kNumXcd;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t stride = (int32_t)(gridDim.x / kNumXcd) * kCellsPerBlock;
    const int64_t ni = DENSE ? nc << shift : nc;
    const int64_t xb = x * items_per_xcd;
    if (xb >= ni) return;
    const int32_t xend = (int32_t)(xb + items_per_xcd < ni ? xb + items_per_xcd : ni);
    int32_t c = (int32_t)xb + kx * kCellsPerBlock + wave;
    if (c >= xend) return;
    const int q0 = lane * V;
    const int32_t sh = DENSE ? shift : 0;
    const int chunk = DENSE ? (c & ((1 << sh) - 1)) : 0;
    const uint32_t cb = (uint32_t)chunk * (uint32_t)(kWave * V * sizeof(T));

    FwdCtx<T> cx;
    cx.row_bytes = (uint32_t)nq * sizeof(T);
    const uint32_t state_bytes = (uint32_t)nc * cx.row_bytes;
    cx.psi = make_rsrc(psi_in, state_bytes);
    cx.out = make_rsrc(psi_out, state_bytes);
    cx.inflow = make_rsrc(a.inflow ? a.inflow : psi_in, a.inflow ? nbf * cx.row_bytes : 0u);
    // no S (a chunked step without scattering): an empty resource, whose loads return 0
    cx.S = make_rsrc(DENSE && S ? S : psi_in, DENSE && S ? state_bytes : 0u);
    // optional per-cell source: read a valid array and scale by 0 when there is none
    cx.src_arr = a.source ? a.source : a.sigma_t;
    cx.src_mul = a.source ? a.dt : T(0);
    cx.inflow_scale = a.inflow_scale;
    cx.dirichlet = a.inflow != nullptr && !a.neumann;
    cx.neumann = a.neumann != 0;
    cx.dpart = dpart;
    // prefetches address the clamped item min(i', xend-1) in [xbeg, xend): always in bounds
    auto clampc = [&](int32_t cc) {
        return uniform_cell((cc < xend ? cc : xend - 1) >> sh);
    };

    const int tq = chunk * kWave * V + q0;      // this lane's first ordinate
    T ox[V], oy[V], wi[V];
    load_slice<V, EXACT>(tab, tq, nq, ox);
    load_slice<V, EXACT>(tab + nq, tq, nq, oy);
    load_slice<V, EXACT>(tab + 3 * nq, tq, nq, wi);
    T w4 = T(0);                                // sum_q w_q / (4 pi), implicit collision only
    if constexpr (IMEX) {
        T part = T(0);
#pragma unroll
        for (int k = 0; k < V; ++k) part += wi[k];
        w4 = cell_sum(part);
    }
    double wd[DOSE ? V : 1];                    // FP64 weights w_q of the fused dose
    if constexpr (DOSE) {
#pragma unroll
        for (int k = 0; k < V; ++k) wd[k] = (EXACT || tq + k < nq) ? wq[tq + k] : 0.0;
    }

    NbrList<MF> n0, n1, n2;
    FwdStage<V, MF, DENSE, T> sa, sb;
    fwd_load_nbr<MF, T>(n0, geom, clampc(c));
    fwd_load_stage<V, EXACT, MF, RHO, DENSE>(sa, n0, geom, clampc(c), cb, nq, q0, a, cx);
    fwd_load_nbr<MF, T>(n1, geom, clampc(c + stride));
    for (;;) {
        // stage B of the next item into sb, stage A of the one after, stage C of this item
        fwd_load_stage<V, EXACT, MF, RHO, DENSE>(sb, n1, geom, clampc(c + stride), cb, nq, q0,
                                                 a, cx);
        fwd_load_nbr<MF, T>(n2, geom, clampc(c + 2 * stride));
        fwd_compute<V, EXACT, MF, RHO, DENSE, T, kAuxStream, IMEX, DOSE>(
            sa, ox, oy, wi, clampc(c), cb, nq, q0, cx, w4, wd, c);
        c += stride;
        if (c >= xend) break;
        n1 = n2;
        fwd_load_stage<V, EXACT, MF, RHO, DENSE>(sa, n1, geom, clampc(c + stride), cb, nq, q0,
                                                 a, cx);
        fwd_load_nbr<MF, T>(n2, geom, clampc(c + 2 * stride));
        fwd_compute<V, EXACT, MF, RHO, DENSE, T, kAuxStream, IMEX, DOSE>(
            sb, ox, oy, wi, clampc(c), cb, nq, q0, cx, w4, wd, c);
        c += stride;
        if (c >= xend) break;
        n1 = n2;
    }
}

template <int V, bool EXACT, int MF, bool RHO, bool DENSE, typename T, bool IMEX = false>
__global__ __launch_bounds__(kStepBlock) void k_step(
    const typename GeomOf<T>::type* __restrict__ geom, int64_t nc, int32_t nq,
    const T* __restrict__ tab, typename ArgsOf<T>::type a, const T* __restrict__ psi_in,
    T* __restrict__ psi_out, const T* __restrict__ S, int64_t items_per_xcd, uint32_t nbf,
    int32_t shift)
{
    step_sweep<V, EXACT, MF, RHO, DENSE, T, IMEX, false>(geom, nc, nq, tab, a, psi_in, psi_out,
                                                         S, items_per_xcd, nbf, shift, nullptr,
                                                         nullptr);
}

// The step with the dose of its input fused: each work item (a row, or one 2^-shift chunk
// of it) also writes dpart[item] = sum_q w_q psi_q over its ordinates in FP64.
template <int V, bool EXACT, int MF, bool RHO, bool DENSE, typename T>
__global__ __launch_bounds__(kStepBlock) void k_step_dose(
    const typename GeomOf<T>::type* __restrict__ geom, int64_t nc, int32_t nq,
    const T* __restrict__ tab, typename ArgsOf<T>::type a, const T* __restrict__ psi_in,
    T* __restrict__ psi_out, const T* __restrict__ S, int64_t items_per_xcd, uint32_t nbf,
    int32_t shift, const double* __restrict__ wq, double* __restrict__ dpart)
{
    step_sweep<V, EXACT, MF, RHO, DENSE, T, false, true>(geom, nc, nq, tab, a, psi_in, psi_out,
                                                         S, items_per_xcd, nbf, shift, wq,
                                                         dpart);
}

// --------------------------------------------------------------------------- adjoint step

// The dense transposed step's update as explicit FMAs (the transposed-step kernels and the
// product tiles of the one-launch transposed step): o = l - cabs l - cstream xs + cscat G
template <int V, typename T>
__device__ __forceinline__ void adj_update(const T (&l)[V], const T (&xs)[V], const T (&g)[V],
                                           T cabs, T cstream, T cscat, T (&o)[V]) {
#pragma unroll
    for (int j = 0; j < V; ++j)
        o[j] = fma_t(cscat, g[j], fma_t(-cstream, xs[j], fma_t(-l[j], cabs, l[j])));
}

// lam_q += coeff (1/rho_c) g_dose[c] w_q in FP64 on an output row of the transposed step (the
// dose functional's term of the reverse rollout, snrt_dose_adjoint's arithmetic).
template <int V, bool EXACT>
__device__ __forceinline__ void dose_adjoint_row(float (&o)[V], const DoseAdj& da,
                                                 const float* __restrict__ inv_rho, int32_t c,
                                                 int q0, int32_t nq) {
    const double g = da.coeff * (inv_rho ? (double)inv_rho[c] : 1.0) * da.g_dose[c];
    double wv[V];
    load_slice<V, EXACT>(da.w, q0, nq, wv);
#pragma unroll
    for (int k = 0; k < V; ++k) o[k] = (float)__builtin_fma(g, wv[k], (double)o[k]);
}

// Adjoint for wide rows (more than 32 bytes of each row per lane, where the pipelined form
// below would hold two stages of them in registers): one wavefront per cell.  GT is the type
// of the gradient accumulators (T, or double so that long runs accumulate in FP64).
// DA: the dose functional's term (dose_adjoint_row) on the output rows (FP32 state, FP64
// gradients only)
template <int V, bool EXACT, bool DENSE, typename T, typename GT = T, bool DA = false>
__global__ __launch_bounds__(kStepBlock) void k_adjoint(
    const typename GeomOf<T>::type* __restrict__ geom, int64_t nc, int32_t mf, int32_t nq,
    const T* __restrict__ tab, typename ArgsOf<T>::type a, const T* __restrict__ psi_n,
    const T* __restrict__ lam_np1, T* __restrict__ lam_n, GT* __restrict__ g_t,
    GT* __restrict__ g_s, GT* __restrict__ g_r, const T* __restrict__ G, DoseAdj da)
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
            if constexpr (DENSE) {
                // the explicit FMAs of adj_downwind_sum
                const T s = fma_t(nx, ox[j], ny * oy[j]);
                const T d = fma_t(-ln[f][j], ia_n[f], l[j] * ia);
                x[j] = (s > T(0) || all_signs) ? fma_t(s, d, x[j]) : x[j];
            } else {
                const T s = ox[j] * nx + oy[j] * ny;
                const T d = l[j] * ia - ln[f][j] * ia_n[f];
                x[j] += (s > T(0) || all_signs) ? s * d : T(0);
            }
        }
    }

    const T irho = a.inv_rho ? a.inv_rho[c] : T(1);
    const T cabs = a.dt * a.alpha_t * a.sigma_t[c];
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
    if constexpr (DENSE) adj_update(l, x, src, cabs, cstream, cscat, o);
#pragma unroll
    for (int j = 0; j < V; ++j) {
        if constexpr (!DENSE) o[j] = (l[j] - cabs * l[j]) - cstream * x[j] + cscat * src[j];
        part_t += l[j] * p[j];
        part_r += p[j] * x[j];
    }
    if constexpr (DA) dose_adjoint_row<V, EXACT>(o, da, a.inv_rho, (int32_t)c, q0, nq);
    store_slice<V, EXACT>(lam_n + c * (int64_t)nq, q0, nq, o);

    if (g_t) {
        const T s = wave_sum(part_t);
        if (lane == 0) g_t[c] += (GT)(-a.dt * a.alpha_t * s);
    }
    if (g_s) {
        const T s = wave_sum(part_s);
        if (lane == 0) g_s[c] += (GT)(a.dt * a.alpha_s * s);
    }
    if (g_r) {
        const T s = wave_sum(part_r);
        if (lane == 0) g_r[c] += (GT)(a.dt * irho * irho * s);
    }
}

// The adjoint step in the persistent, XCD-partitioned, pipelined form of the forward
// sweep: stage B loads the next cell's rows (own lambda and psi, each face's lambda, the
// neighbours' 1/A, the dense G row) while stage C computes this one.  Faces are branch-free:
// interior faces (and the zero-normal self-faces of unused slots) read the neighbour's
// lambda with its 1/A, boundary faces the cell's own row with weight 0; a Neumann boundary
// face passes both flux signs (its ghost is the cell's own value).
template <int V, int MF, bool DENSE, typename T, typename GT>
struct AdjStage {
    T l[V], p[V];
    T ln[MF][V];
    T g[DENSE ? V : 1];
    T ia_n[MF], nx[MF], ny[MF];
    bool all_signs[MF];
    T ia, irho, cabs, cscat;
    GT gt0, gs0, gr0;               // the gradient accumulators' values before this step
};

template <typename T, typename GT>
struct AdjCtx {
    __amdgpu_buffer_rsrc_t lam, psi, out, G;
    uint32_t row_bytes;
    bool neumann;
    GT *g_t, *g_s, *g_r;
    DoseAdj da;       // the dose functional's term of a reverse rollout (g_dose NULL: none)
};


// The dense transposed step's downwind sum as explicit FMAs (shared by the transposed-step
// kernels and the product tiles of the one-launch transposed step):
//   xs = sum_f [s_f > 0 or Neumann ghost] s_f (l/A - l_f/A_f),   s_f = Omega . n_f
template <int V, int MF, bool DENSE, typename T, typename GT>
__device__ __forceinline__ void adj_downwind_sum(const AdjStage<V, MF, DENSE, T, GT>& d,
                                                 const T (&ox)[V], const T (&oy)[V],
                                                 T (&xs)[V]) {
#pragma unroll
    for (int f = 0; f < MF; ++f) {
#pragma unroll
        for (int j = 0; j < V; ++j) {
            const T s = fma_t(d.nx[f], ox[j], d.ny[f] * oy[j]);
            const T dd = fma_t(-d.ln[f][j], d.ia_n[f], d.l[j] * d.ia);
            xs[j] = (s > T(0) || d.all_signs[f]) ? fma_t(s, dd, xs[j]) : xs[j];
        }
    }
}

template <int V, bool EXACT, int MF, bool DENSE, typename T, typename GT>
__device__ __forceinline__ void adj_load_stage(AdjStage<V, MF, DENSE, T, GT>& d,
                                               const NbrList<MF>& nb,
                                               const typename GeomOf<T>::type* __restrict__ geom,
                                               int32_t c, int32_t nq, int q0,
                                               const typename ArgsOf<T>::type& a,
                                               const AdjCtx<T, GT>& x)
{
    const auto* g = cell_rec(geom, c);
    const uint32_t own = (uint32_t)c * x.row_bytes;
    buf_load_row<V, EXACT, T>(x.lam, own, q0, nq, d.l);
    buf_load_row<V, EXACT, T>(x.psi, own, q0, nq, d.p);
#pragma unroll
    for (int f = 0; f < MF; ++f) {
        const int32_t j = nb.j[f];
        const bool interior = j >= 0;
        const int32_t src = uniform_cell(interior ? j : c);
        buf_load_row<V, EXACT, T>(x.lam, (uint32_t)src * x.row_bytes, q0, nq, d.ln[f]);
        d.ia_n[f] = interior ? cell_rec(geom, src)->inv_area : T(0);
        d.all_signs[f] = !interior && x.neumann;
        d.nx[f] = g->n[f][0];
        d.ny[f] = g->n[f][1];
    }
    if constexpr (DENSE) buf_load_row<V, EXACT, T>(x.G, own, q0, nq, d.g);
    d.ia = g->inv_area;
    d.irho = a.inv_rho ? cell_val(a.inv_rho, c) : T(1);
    d.cabs = a.dt * a.alpha_t * cell_val(a.sigma_t, c);
    d.cscat = a.dt * a.alpha_s * cell_val(a.sigma_s, c);
    // each cell's accumulators are updated once per launch (by this wavefront), so their
    // old values can be fetched a stage ahead instead of stalling the update on the load
    d.gt0 = x.g_t ? cell_val(x.g_t, c) : GT(0);
    d.gs0 = x.g_s ? cell_val(x.g_s, c) : GT(0);
    d.gr0 = x.g_r ? cell_val(x.g_r, c) : GT(0);
}

template <int V, bool EXACT, int MF, bool DENSE, typename T, typename GT, bool DA = false>
__device__ __forceinline__ void adj_compute(const AdjStage<V, MF, DENSE, T, GT>& d,
                                            const T (&ox)[V], const T (&oy)[V],
                                            const T (&wi)[V], int32_t c, int32_t nq, int q0,
                                            int lane, const typename ArgsOf<T>::type& a,
                                            const AdjCtx<T, GT>& x)
{
    T xs[V];
#pragma unroll
    for (int j = 0; j < V; ++j) xs[j] = T(0);
    if constexpr (DENSE) {
        // explicit FMAs (as in the dense forward update): the same bits wherever inlined
        adj_downwind_sum(d, ox, oy, xs);
    } else {
#pragma unroll
        for (int f = 0; f < MF; ++f) {
#pragma unroll
            for (int j = 0; j < V; ++j) {
                const T s = ox[j] * d.nx[f] + oy[j] * d.ny[f];
                const T dd = d.l[j] * d.ia - d.ln[f][j] * d.ia_n[f];
                xs[j] += (s > T(0) || d.all_signs[f]) ? s * dd : T(0);
            }
        }
    }
    const T cstream = a.dt * d.irho;
    T src[V];
    T part_s;                                     // per-lane part of sum_q l_q S_q
    if constexpr (DENSE) {
        part_s = T(0);
#pragma unroll
        for (int j = 0; j < V; ++j) {
            src[j] = d.g[j];                      // (Lambda B^T)_cq
            part_s += d.p[j] * src[j];
        }
    } else {
        T pl = T(0), pw = T(0);
#pragma unroll
        for (int j = 0; j < V; ++j) {
            pl += d.l[j];
            pw += wi[j] * d.p[j];
        }
        const T lsum = cell_sum(pl);
        const T scell = cell_sum(pw);             // isotropic S of the cell
#pragma unroll
        for (int j = 0; j < V; ++j) src[j] = wi[j] * lsum;
        part_s = (lane == 0) ? scell * lsum : T(0);
    }
    T o[V];
    T part_t = T(0), part_r = T(0);
    if constexpr (DENSE) {
        adj_update(d.l, xs, src, d.cabs, cstream, d.cscat, o);
#pragma unroll
        for (int j = 0; j < V; ++j) {
            part_t += d.l[j] * d.p[j];
            part_r += d.p[j] * xs[j];
        }
    } else {
#pragma unroll
        for (int j = 0; j < V; ++j) {
            o[j] = (d.l[j] - d.cabs * d.l[j]) - cstream * xs[j] + d.cscat * src[j];
            part_t += d.l[j] * d.p[j];
            part_r += d.p[j] * xs[j];
        }
    }
    if constexpr (DA) dose_adjoint_row<V, EXACT>(o, x.da, a.inv_rho, c, q0, nq);
    buf_store_row<V, EXACT, T, kAuxStream>(x.out, (uint32_t)c * x.row_bytes, q0, nq, o);
    if (x.g_t) {
        const T s = cell_sum(part_t);
        if (lane == 0) x.g_t[c] = d.gt0 + (GT)(-a.dt * a.alpha_t * s);
    }
    if (x.g_s) {
        const T s = cell_sum(part_s);
        if (lane == 0) x.g_s[c] = d.gs0 + (GT)(a.dt * a.alpha_s * s);
    }
    if (x.g_r) {
        const T s = cell_sum(part_r);
        if (lane == 0) x.g_r[c] = d.gr0 + (GT)(a.dt * d.irho * d.irho * s);
    }
}

template <int V, bool EXACT, int MF, bool DENSE, typename T, typename GT = T, bool DA = false>
__global__ __launch_bounds__(kStepBlock) void k_adjoint_p(
    const typename GeomOf<T>::type* __restrict__ geom, int64_t nc, int32_t nq,
    const T* __restrict__ tab, typename ArgsOf<T>::type a, const T* __restrict__ psi_n,
    const T* __restrict__ lam_np1, T* __restrict__ lam_n, GT* __restrict__ g_t,
    GT* __restrict__ g_s, GT* __restrict__ g_r, const T* __restrict__ G, int64_t items_per_xcd,
    DoseAdj da)
{
    const int x = blockIdx.x % kNumXcd;
    const int kx = blockIdx.x / kNumXcd;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t stride = (int32_t)(gridDim.x / kNumXcd) * kCellsPerBlock;
    const int64_t xb = x * items_per_xcd;
    if (xb >= nc) return;
    const int32_t xend = (int32_t)(xb + items_per_xcd < nc ? xb + items_per_xcd : nc);
    int32_t c = (int32_t)xb + kx * kCellsPerBlock + wave;
    if (c >= xend) return;
    const int q0 = lane * V;

    AdjCtx<T, GT> cx;
    cx.row_bytes = (uint32_t)nq * sizeof(T);
    const uint32_t state_bytes = (uint32_t)nc * cx.row_bytes;
    cx.lam = make_rsrc(lam_np1, state_bytes);
    cx.psi = make_rsrc(psi_n, state_bytes);
    cx.out = make_rsrc(lam_n, state_bytes);
    cx.G = make_rsrc(DENSE ? G : lam_np1, DENSE ? state_bytes : 0u);
    cx.neumann = a.neumann != 0;
    cx.g_t = g_t;
    cx.g_s = g_s;
    cx.g_r = g_r;
    cx.da = da;
    // prefetches address the clamped cell min(c', xend-1): always in bounds
    auto clampc = [xend](int32_t cc) { return uniform_cell(cc < xend ? cc : xend - 1); };

    T ox[V], oy[V], wi[V];
    load_slice<V, EXACT>(tab, q0, nq, ox);
    load_slice<V, EXACT>(tab + nq, q0, nq, oy);
    load_slice<V, EXACT>(tab + 3 * nq, q0, nq, wi);

    NbrList<MF> n0, n1, n2;
    AdjStage<V, MF, DENSE, T, GT> sa, sb;
    fwd_load_nbr<MF, T>(n0, geom, clampc(c));
    adj_load_stage<V, EXACT, MF, DENSE>(sa, n0, geom, clampc(c), nq, q0, a, cx);
    fwd_load_nbr<MF, T>(n1, geom, clampc(c + stride));
    for (;;) {
        adj_load_stage<V, EXACT, MF, DENSE>(sb, n1, geom, clampc(c + stride), nq, q0, a, cx);
        fwd_load_nbr<MF, T>(n2, geom, clampc(c + 2 * stride));
        adj_compute<V, EXACT, MF, DENSE, T, GT, DA>(sa, ox, oy, wi, clampc(c), nq, q0, lane, a,
                                                    cx);
        c += stride;
        if (c >= xend) break;
        n1 = n2;
        adj_load_stage<V, EXACT, MF, DENSE>(sa, n1, geom, clampc(c + stride), nq, q0, a, cx);
        fwd_load_nbr<MF, T>(n2, geom, clampc(c + 2 * stride));
        adj_compute<V, EXACT, MF, DENSE, T, GT, DA>(sb, ox, oy, wi, clampc(c), nq, q0, lane, a,
                                                    cx);
        c += stride;
        if (c >= xend) break;
        n1 = n2;
    }
}

// --------------------------------------------------------------------------- dispatch helpers

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

// Launch shape of the persistent step: ``blocks_per_cu`` resident 4-wave blocks per CU
// (rounded to the XCD count), never more blocks than there are CPW-cell groups.
struct StepShape {
    unsigned blocks;
    int64_t cells_per_xcd;
};

inline StepShape step_shape(const snrt_mesh& m, int64_t items, int cpw,
                            int resident_blocks_per_cu, int blocks_per_cu = 0) {
    int bpc = blocks_per_cu > 0 ? blocks_per_cu : tune().step_blocks_per_cu;
    if (resident_blocks_per_cu > 0 && bpc > resident_blocks_per_cu) bpc = resident_blocks_per_cu;
    int64_t want = (items + (int64_t)kCellsPerBlock - 1) / (int64_t)kCellsPerBlock;
    int64_t cap = (int64_t)m.num_cu * bpc;
    int64_t b = want < cap ? want : cap;
    b = (b / kNumXcd) * kNumXcd;             // equal block count per XCD, never above cap
    if (b < kNumXcd) b = kNumXcd;
    int64_t cpx = (items + kNumXcd - 1) / kNumXcd;
    cpx = ((cpx + cpw - 1) / cpw) * cpw;     // a multiple of cpw items per XCD
    return {(unsigned)b, cpx};
}

// Blocks of a kernel that fit on one CU at once (registers / LDS), queried once.  A
// persistent grid larger than this would run its last blocks after the others finish.
template <typename K>
int resident_blocks(K kernel) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, kStepBlock, 0) != hipSuccess)
        n = 0;
    return n;
}

template <typename T, int V, bool E, int MF, bool RHO, bool DENSE, bool IMEX = false>
hipError_t launch_fwd(const typename GeomOf<T>::type* geom, const snrt_mesh& m, const T* tab,
                      int32_t nq, const typename ArgsOf<T>::type& a, const T* psi_in,
                      T* psi_out, const T* S, int shift, hipStream_t st,
                      const double* wq = nullptr, double* dpart = nullptr)
{
    if (dpart) {
        if constexpr (!IMEX) {
            static const int occ = resident_blocks(k_step_dose<V, E, MF, RHO, DENSE, T>);
            const StepShape sh = step_shape(m, m.nc << shift, shift ? kCellsPerBlock : 1, occ);
            hipLaunchKernelGGL((k_step_dose<V, E, MF, RHO, DENSE, T>), dim3(sh.blocks),
                               dim3(kStepBlock), 0, st, geom, m.nc, nq, tab, a, psi_in, psi_out,
                               S, sh.cells_per_xcd, (uint32_t)m.nbf, (int32_t)shift, wq, dpart);
            return hipGetLastError();
        }
        return hipErrorNotSupported;
    }
    static const int occ = resident_blocks(k_step<V, E, MF, RHO, DENSE, T, IMEX>);
    const StepShape sh = step_shape(m, m.nc << shift, shift ? kCellsPerBlock : 1, occ);
    hipLaunchKernelGGL((k_step<V, E, MF, RHO, DENSE, T, IMEX>), dim3(sh.blocks), dim3(kStepBlock),
                       0, st, geom, m.nc, nq, tab, a, psi_in, psi_out, S, sh.cells_per_xcd,
                       (uint32_t)m.nbf, (int32_t)shift);
    return hipGetLastError();
}

// Dense scattering with 256-ordinate-multiple rows of 2 or 4 chunks runs as 4-ordinate
// lanes over row chunks; returns the chunk shift (0: whole rows).
inline int dense_chunk_shift(int32_t nq) {
    if (nq == 2 * kWave * 4) return 1;
    if (nq == 4 * kWave * 4) return 2;
    return 0;
}

// Implicit-collision (IMEX) step, isotropic scattering only.
template <typename T>
hipError_t launch_imex_t(const typename GeomOf<T>::type* geom, const snrt_mesh& m,
                         const T* tab, int32_t nq, const typename ArgsOf<T>::type& a,
                         const T* psi_in, T* psi_out, hipStream_t st)
{
    if (m.nc == 0) return hipSuccess;
    const bool rho = a.inv_rho != nullptr, mf4 = m.mf == 4;
    return dispatch_v<T>(nq, [&](auto vc, auto ex) {
        constexpr int V = decltype(vc)::value;
        constexpr bool E = decltype(ex)::value;
        auto go = [&](auto mfc, auto rc) {
            constexpr int MF = decltype(mfc)::value;
            constexpr bool R = decltype(rc)::value;
            return launch_fwd<T, V, E, MF, R, false, true>(geom, m, tab, nq, a, psi_in, psi_out,
                                                           nullptr, 0, st);
        };
        using I3 = std::integral_constant<int, 3>;
        using I4 = std::integral_constant<int, 4>;
        if (mf4) return rho ? go(I4{}, std::true_type{}) : go(I4{}, std::false_type{});
        return rho ? go(I3{}, std::true_type{}) : go(I3{}, std::false_type{});
    });
}

template <typename T>
hipError_t launch_step_t(const typename GeomOf<T>::type* geom, const snrt_mesh& m,
                         const T* tab, int32_t nq, const typename ArgsOf<T>::type& a,
                         const T* psi_in, T* psi_out, const T* S, hipStream_t st,
                         const double* wq = nullptr, double* dpart = nullptr,
                         bool chunk_rows = false)
{
    if (m.nc == 0) return hipSuccess;
    // chunk_rows without S: the chunked (dense-row) kernel with a zero scattering source, for
    // steps that need no in-row reduction
    const bool rho = a.inv_rho != nullptr, dense = S != nullptr || chunk_rows, mf4 = m.mf == 4;
    const int shift = dense ? dense_chunk_shift(nq) : 0;
    return dispatch_v<T>(shift ? kWave * 4 : nq, [&](auto vc, auto ex) {
        constexpr int V = decltype(vc)::value;
        constexpr bool E = decltype(ex)::value;
        auto go = [&](auto mfc, auto rc, auto dc) {
            constexpr int MF = decltype(mfc)::value;
            constexpr bool R = decltype(rc)::value;
            constexpr bool D = decltype(dc)::value;
            return launch_fwd<T, V, E, MF, R, D>(geom, m, tab, nq, a, psi_in, psi_out, S,
                                                 shift, st, wq, dpart);
        };
        using I3 = std::integral_constant<int, 3>;
        using I4 = std::integral_constant<int, 4>;
        using Tt = std::true_type;
        using Ff = std::false_type;
        if (!mf4) {
            if (rho) return dense ? go(I3{}, Tt{}, Tt{}) : go(I3{}, Tt{}, Ff{});
            return dense ? go(I3{}, Ff{}, Tt{}) : go(I3{}, Ff{}, Ff{});
        }
        if (rho) return dense ? go(I4{}, Tt{}, Tt{}) : go(I4{}, Tt{}, Ff{});
        return dense ? go(I4{}, Ff{}, Tt{}) : go(I4{}, Ff{}, Ff{});
    });
}

template <typename T, typename GT = T>
hipError_t launch_adjoint_t(const typename GeomOf<T>::type* geom, const snrt_mesh& m,
                            const T* tab, int32_t nq, const typename ArgsOf<T>::type& a,
                            const T* psi_n, const T* lam_np1, T* lam_n, GT* g_t, GT* g_s,
                            GT* g_r, const T* G, hipStream_t st, const DoseAdj& da = DoseAdj())
{
    if (m.nc == 0) return hipSuccess;
    constexpr bool kCanDA = std::is_same<T, float>::value && std::is_same<GT, double>::value;
    if (da.g_dose && !kCanDA) return hipErrorInvalidValue;
    auto with_da = [&](auto da_c) {
        constexpr bool DA = decltype(da_c)::value;
        return dispatch_v<T>(nq, [&](auto vc, auto ex) {
            constexpr int V = decltype(vc)::value;
            constexpr bool E = decltype(ex)::value;
            if constexpr (V * sizeof(T) > 32) {
                const unsigned blocks = (unsigned)((m.nc + kCellsPerBlock - 1) / kCellsPerBlock);
                if (G)
                    hipLaunchKernelGGL((k_adjoint<V, E, true, T, GT, DA>), dim3(blocks),
                                       dim3(kStepBlock), 0, st, geom, m.nc, m.mf, nq, tab, a,
                                       psi_n, lam_np1, lam_n, g_t, g_s, g_r, G, da);
                else
                    hipLaunchKernelGGL((k_adjoint<V, E, false, T, GT, DA>), dim3(blocks),
                                       dim3(kStepBlock), 0, st, geom, m.nc, m.mf, nq, tab, a,
                                       psi_n, lam_np1, lam_n, g_t, g_s, g_r, G, da);
                return hipGetLastError();
            } else {
                auto go = [&](auto mfc, auto dc) {
                    constexpr int MF = decltype(mfc)::value;
                    constexpr bool D = decltype(dc)::value;
                    static const int occ = resident_blocks(k_adjoint_p<V, E, MF, D, T, GT, DA>);
                    const StepShape sh =
                        step_shape(m, m.nc, 1, occ, tune().adjoint_blocks_per_cu);
                    hipLaunchKernelGGL((k_adjoint_p<V, E, MF, D, T, GT, DA>), dim3(sh.blocks),
                                       dim3(kStepBlock), 0, st, geom, m.nc, nq, tab, a, psi_n,
                                       lam_np1, lam_n, g_t, g_s, g_r, G, sh.cells_per_xcd, da);
                    return hipGetLastError();
                };
                using I3 = std::integral_constant<int, 3>;
                using I4 = std::integral_constant<int, 4>;
                if (m.mf == 4)
                    return G ? go(I4{}, std::true_type{}) : go(I4{}, std::false_type{});
                return G ? go(I3{}, std::true_type{}) : go(I3{}, std::false_type{});
            }
        });
    };
    if constexpr (kCanDA) {
        if (da.g_dose) return with_da(std::true_type{});
    }
    return with_da(std::false_type{});
}

}  // namespace snrt
