// Second-order scheme (Sec. 4.2, second order finite volume schemes): per stage, a limited
// Green-Gauss gradient of u = psi/rho, then the explicit Euler update whose upwind flux takes
// linear reconstructions of u on both sides of every face.  The host runs two stages and
// averages (Heun).
//
// k_grad2 (one wavefront per cell or per 256-ordinate chunk of a cell, lane = V ordinates):
//   grad u_i = 1/A_i sum_f (u_i + u_f)/2 n_if          (u_f: neighbour value or ghost value)
//   Psi_i    = min_f phi(d1_f, d_f), d_f = grad u_i . r_if, d1_f = u_max - u_i if d_f > 0,
//              u_min - u_i if d_f < 0 (u_max/u_min over u_i and every u_f), phi = 1 at d_f = 0;
//              Barth-Jespersen: phi = min(1, d1/d);  Venkatakrishnan:
//              phi = (d1^2 + eps^2 + 2 d d1) / (d1^2 + 2 d^2 + d d1 + eps^2),
//              eps^2 = (K sqrt(A_i))^3 (the d-divided form of the smooth limiter)
//   G_i      = Psi_i grad u_i, stored as two rows per cell: [cell][x|y][nq].
// k_flux2 (one wavefront per cell; k_flux2p is the same update in the persistent,
// pipelined form of the first-order step, used whenever the gradient fits 32-bit offsets):
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

template <int V, bool EXACT, int MF, bool RHO, int LIM, typename T>
__global__ __launch_bounds__(kStepBlock) void k_grad2(
    const typename GeomOf<T>::type* __restrict__ geom,
    const typename ReconOf<T>::type* __restrict__ recon, int64_t nc, int32_t nq,
    typename ArgsOf<T>::type a, const T* __restrict__ psi, T* __restrict__ G, int32_t shift,
    T vk_k)
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
    T eps2 = T(0);
    if constexpr (LIM == SNRT_LIMITER_VENKATAKRISHNAN) {
        const T h = vk_k * sqrt(T(1) / g.inv_area);
        eps2 = h * h * h;
    }
#pragma unroll
    for (int f = 0; f < MF; ++f) {
        const T rx = rc.r_own[f][0], ry = rc.r_own[f][1];
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const T d2 = gx[k] * rx + gy[k] * ry;
            const T d1 = d2 > T(0) ? umax[k] - u[k] : umin[k] - u[k];
            T t = T(1);
            if constexpr (LIM == SNRT_LIMITER_VENKATAKRISHNAN) {
                // d1 d2 >= 0, so the denominator is at least 2 d2^2 > 0 whenever d2 != 0
                const T d11 = d1 * d1 + eps2;
                if (d2 != T(0)) t = (d11 + T(2) * d2 * d1) / (d11 + T(2) * d2 * d2 + d1 * d2);
            } else {
                if (d2 != T(0)) t = d1 / d2;
                t = t < T(1) ? t : T(1);
            }
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

    const T cabs = a.dt * a.alpha_t * a.sigma_t[c];   // absorption as p - cabs p
    const T cflux = a.dt * g.inv_area;
    const T cscat = a.dt * a.alpha_s * a.sigma_s[c];
    const T csrc = a.source ? a.dt * a.source[c] : T(0);
    T o[V];
#pragma unroll
    for (int k = 0; k < V; ++k) o[k] = (p[k] - cabs * p[k]) - cflux * acc[k] + cscat * src[k] + csrc;
    if constexpr (FINAL) {
        T pn[V];
        load_slice<V, EXACT>(psi_n + c * nq, q0, nq, pn);
#pragma unroll
        for (int k = 0; k < V; ++k) o[k] = T(0.5) * (pn[k] + o[k]);
    }
    store_slice<V, EXACT>(out + c * nq, q0, nq, o);
}

// --------------------------------------------------------------- persistent stage update
// The same update as k_flux2 in the persistent, XCD-partitioned, software-pipelined form of
// the first-order step kernel: every wave sweeps a contiguous item range of its XCD, loading
// the next cell's rows (own psi and G, each face's far-side psi and G) while it computes the
// current one.  Requires the gradient array below 4 GiB.

template <int V, int MF, bool DENSE, bool FINAL, typename T>
struct Flux2Stage {
    T p[V], gx[V], gy[V];
    T up[MF][V], gxj[MF][V], gyj[MF][V];
    T src[V], pn[V];
    T ghost[MF];
    T nx[MF], ny[MF], rox[MF], roy[MF], rfx[MF], rfy[MF];
    T irho, cabs, cflux, cscat, csrc;
};

template <typename T>
struct Flux2Ctx {
    __amdgpu_buffer_rsrc_t psi, G, inflow, out, S, pn;
    uint32_t row_bytes;
    const T* src_arr;
    T src_mul, inflow_scale;
    bool dirichlet, neumann;
};

template <int V, bool EXACT, int MF, bool RHO, bool DENSE, bool FINAL, typename T>
__device__ __forceinline__ void flux2_load(Flux2Stage<V, MF, DENSE, FINAL, T>& d,
                                           const NbrList<MF>& nb,
                                           const typename GeomOf<T>::type* __restrict__ geom,
                                           const typename ReconOf<T>::type* __restrict__ recon,
                                           int32_t c, uint32_t cb, int32_t nq, int q0,
                                           const typename ArgsOf<T>::type& a,
                                           const Flux2Ctx<T>& x)
{
    const auto* g = cell_rec(geom, c);
    const auto* rc = cell_rec(recon, c);
    const uint32_t own = (uint32_t)c * x.row_bytes + cb;
    const uint32_t gown = 2u * (uint32_t)c * x.row_bytes + cb;
    buf_load_row<V, EXACT, T>(x.psi, own, q0, nq, d.p);
    buf_load_row<V, EXACT, T>(x.G, gown, q0, nq, d.gx);
    buf_load_row<V, EXACT, T>(x.G, gown + x.row_bytes, q0, nq, d.gy);
    d.irho = RHO ? cell_val(a.inv_rho, c) : T(1);
    const T bscale = x.dirichlet ? x.inflow_scale : (x.neumann ? d.irho : T(0));
#pragma unroll
    for (int f = 0; f < MF; ++f) {
        const int32_t j = nb.j[f];
        const bool bnd = j < 0;
        const int32_t bidx = x.dirichlet ? -1 - j : c;
        const uint32_t off = (uint32_t)(bnd ? bidx : j) * x.row_bytes + cb;
        const T rho_j = RHO ? cell_val(a.inv_rho, bnd ? c : j) : T(1);
        d.ghost[f] = bnd ? bscale : rho_j;
        buf_load_row<V, EXACT, T>(bnd && x.dirichlet ? x.inflow : x.psi, off, q0, nq, d.up[f]);
        // r_far is zero on boundary faces and unused slots: their own G rows are read and
        // multiplied by zero
        const uint32_t goff = 2u * (uint32_t)(bnd ? c : j) * x.row_bytes + cb;
        buf_load_row<V, EXACT, T>(x.G, goff, q0, nq, d.gxj[f]);
        buf_load_row<V, EXACT, T>(x.G, goff + x.row_bytes, q0, nq, d.gyj[f]);
        d.nx[f] = g->n[f][0];
        d.ny[f] = g->n[f][1];
        d.rox[f] = rc->r_own[f][0];
        d.roy[f] = rc->r_own[f][1];
        d.rfx[f] = rc->r_far[f][0];
        d.rfy[f] = rc->r_far[f][1];
    }
    if constexpr (DENSE) buf_load_row<V, EXACT, T>(x.S, own, q0, nq, d.src);
    if constexpr (FINAL) buf_load_row<V, EXACT, T>(x.pn, own, q0, nq, d.pn);
    d.cabs = a.dt * a.alpha_t * cell_val(a.sigma_t, c);
    d.cflux = a.dt * g->inv_area;
    d.cscat = a.dt * a.alpha_s * cell_val(a.sigma_s, c);
    d.csrc = x.src_mul * cell_val(x.src_arr, c);
}

template <int V, bool EXACT, int MF, bool RHO, bool DENSE, bool FINAL, typename T>
__device__ __forceinline__ void flux2_compute(const Flux2Stage<V, MF, DENSE, FINAL, T>& d,
                                              const T (&ox)[V], const T (&oy)[V],
                                              const T (&wi)[V], int32_t c, uint32_t cb,
                                              int32_t nq, int q0, const Flux2Ctx<T>& x)
{
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
#pragma unroll
    for (int f = 0; f < MF; ++f) {
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const T s = ox[k] * d.nx[f] + oy[k] * d.ny[f];
            const T ui = u[k] + d.gx[k] * d.rox[f] + d.gy[k] * d.roy[f];
            const T uj = d.up[f][k] * d.ghost[f] + d.gxj[f][k] * d.rfx[f] + d.gyj[f][k] * d.rfy[f];
            acc[k] += (s > T(0)) ? s * ui : s * uj;
        }
    }
    T o[V];
#pragma unroll
    for (int k = 0; k < V; ++k) {
        o[k] = (d.p[k] - d.cabs * d.p[k]) - d.cflux * acc[k] + d.cscat * src[k] + d.csrc;
        if constexpr (FINAL) o[k] = T(0.5) * (d.pn[k] + o[k]);
    }
    buf_store_row<V, EXACT, T, kAuxStream>(x.out, (uint32_t)c * x.row_bytes + cb, q0, nq, o);
}

template <int V, bool EXACT, int MF, bool RHO, bool DENSE, bool FINAL, typename T>
__global__ __launch_bounds__(kStepBlock) void k_flux2p(
    const typename GeomOf<T>::type* __restrict__ geom,
    const typename ReconOf<T>::type* __restrict__ recon, int64_t nc, int32_t nq,
    const T* __restrict__ tab, typename ArgsOf<T>::type a, const T* __restrict__ psi,
    const T* __restrict__ G, const T* __restrict__ S, const T* __restrict__ psi_n,
    T* __restrict__ out, int64_t items_per_xcd, uint32_t nbf, int32_t shift)
{
    const int x = blockIdx.x % kNumXcd;
    const int kx = blockIdx.x / kNumXcd;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t stride = (int32_t)(gridDim.x / kNumXcd) * kCellsPerBlock;
    const int64_t ni = nc << shift;
    const int64_t xb = x * items_per_xcd;
    if (xb >= ni) return;
    const int32_t xend = (int32_t)(xb + items_per_xcd < ni ? xb + items_per_xcd : ni);
    int32_t c = (int32_t)xb + kx * kCellsPerBlock + wave;
    if (c >= xend) return;
    const int q0 = lane * V;
    const int32_t sh = shift;
    const int chunk = c & ((1 << sh) - 1);
    const uint32_t cb = (uint32_t)chunk * (uint32_t)(kWave * V * sizeof(T));

    Flux2Ctx<T> cx;
    cx.row_bytes = (uint32_t)nq * sizeof(T);
    const uint32_t state_bytes = (uint32_t)nc * cx.row_bytes;
    cx.psi = make_rsrc(psi, state_bytes);
    cx.G = make_rsrc(G, 2u * state_bytes);
    cx.out = make_rsrc(out, state_bytes);
    cx.inflow = make_rsrc(a.inflow ? a.inflow : psi, a.inflow ? nbf * cx.row_bytes : 0u);
    cx.S = make_rsrc(DENSE ? S : psi, DENSE ? state_bytes : 0u);
    cx.pn = make_rsrc(FINAL ? psi_n : psi, FINAL ? state_bytes : 0u);
    cx.src_arr = a.source ? a.source : a.sigma_t;
    cx.src_mul = a.source ? a.dt : T(0);
    cx.inflow_scale = a.inflow_scale;
    cx.dirichlet = a.inflow != nullptr && !a.neumann;
    cx.neumann = a.neumann != 0;
    // prefetches address the clamped item min(i', xend-1) in [xbeg, xend): always in bounds
    auto clampc = [xend, sh](int32_t cc) {
        return uniform_cell((cc < xend ? cc : xend - 1) >> sh);
    };

    const int tq = chunk * kWave * V + q0;
    T ox[V], oy[V], wi[V];
    load_slice<V, EXACT>(tab, tq, nq, ox);
    load_slice<V, EXACT>(tab + nq, tq, nq, oy);
    load_slice<V, EXACT>(tab + 3 * nq, tq, nq, wi);

    NbrList<MF> n0, n1, n2;
    Flux2Stage<V, MF, DENSE, FINAL, T> sa, sb;
    fwd_load_nbr<MF, T>(n0, geom, clampc(c));
    flux2_load<V, EXACT, MF, RHO>(sa, n0, geom, recon, clampc(c), cb, nq, q0, a, cx);
    fwd_load_nbr<MF, T>(n1, geom, clampc(c + stride));
    for (;;) {
        flux2_load<V, EXACT, MF, RHO>(sb, n1, geom, recon, clampc(c + stride), cb, nq, q0, a, cx);
        fwd_load_nbr<MF, T>(n2, geom, clampc(c + 2 * stride));
        flux2_compute<V, EXACT, MF, RHO>(sa, ox, oy, wi, clampc(c), cb, nq, q0, cx);
        c += stride;
        if (c >= xend) break;
        n1 = n2;
        flux2_load<V, EXACT, MF, RHO>(sa, n1, geom, recon, clampc(c + stride), cb, nq, q0, a, cx);
        fwd_load_nbr<MF, T>(n2, geom, clampc(c + 2 * stride));
        flux2_compute<V, EXACT, MF, RHO>(sb, ox, oy, wi, clampc(c), cb, nq, q0, cx);
        c += stride;
        if (c >= xend) break;
        n1 = n2;
    }
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
                          const typename ArgsOf<T>::type& a, const Limiter& lim, const T* psi,
                          T* G, const typename GeomOf<T>::type* geom,
                          const typename ReconOf<T>::type* recon, hipStream_t st)
{
    if (m.nc == 0) return hipSuccess;
    const int shift = chunk_shift(q.nq);
    const bool rho = a.inv_rho != nullptr, mf4 = m.mf == 4;
    const bool vk = lim.kind == SNRT_LIMITER_VENKATAKRISHNAN;
    return dispatch_v<T>(shift ? kWave * 4 : q.nq, [&](auto vc, auto ex) {
        constexpr int V = decltype(vc)::value;
        constexpr bool E = decltype(ex)::value;
        auto go = [&](auto mfc, auto rcst, auto lc) {
            constexpr int MF = decltype(mfc)::value;
            constexpr bool R = decltype(rcst)::value;
            constexpr int L = decltype(lc)::value;
            hipLaunchKernelGGL((k_grad2<V, E, MF, R, L, T>), dim3(item_blocks(m.nc, shift)),
                               dim3(kStepBlock), 0, st, geom, recon, m.nc, q.nq, a, psi, G,
                               (int32_t)shift, (T)lim.k);
            return hipGetLastError();
        };
        auto by_lim = [&](auto mfc, auto rcst) {
            return vk ? go(mfc, rcst, std::integral_constant<int, SNRT_LIMITER_VENKATAKRISHNAN>{})
                      : go(mfc, rcst, std::integral_constant<int, SNRT_LIMITER_BARTH_JESPERSEN>{});
        };
        using I3 = std::integral_constant<int, 3>;
        using I4 = std::integral_constant<int, 4>;
        if (mf4) return rho ? by_lim(I4{}, std::true_type{}) : by_lim(I4{}, std::false_type{});
        return rho ? by_lim(I3{}, std::true_type{}) : by_lim(I3{}, std::false_type{});
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
    // the persistent kernel addresses the gradient (two rows per cell) with 32-bit offsets
    const bool persistent = 2 * m.nc * (int64_t)q.nq * (int64_t)sizeof(T) < (int64_t(1) << 32);
    return dispatch_v<T>(shift ? kWave * 4 : q.nq, [&](auto vc, auto ex) {
        constexpr int V = decltype(vc)::value;
        constexpr bool E = decltype(ex)::value;
        auto go = [&](auto mfc, auto rcst, auto dcst, auto fcst) {
            constexpr int MF = decltype(mfc)::value;
            constexpr bool R = decltype(rcst)::value;
            constexpr bool D = decltype(dcst)::value;
            constexpr bool F = decltype(fcst)::value;
            if (persistent) {
                static const int occ = resident_blocks(k_flux2p<V, E, MF, R, D, F, T>);
                const StepShape sp = step_shape(m, m.nc << shift, shift ? kCellsPerBlock : 1, occ,
                                                tune().flux2_blocks_per_cu);
                hipLaunchKernelGGL((k_flux2p<V, E, MF, R, D, F, T>), dim3(sp.blocks),
                                   dim3(kStepBlock), 0, st, geom, recon, m.nc, q.nq, tab, a, psi,
                                   G, S, psi_n, out, sp.cells_per_xcd, (uint32_t)m.nbf,
                                   (int32_t)shift);
            } else {
                hipLaunchKernelGGL((k_flux2<V, E, MF, R, D, F, T>), dim3(item_blocks(m.nc, shift)),
                                   dim3(kStepBlock), 0, st, geom, recon, m.nc, q.nq, tab, a, psi,
                                   G, S, psi_n, out, (int32_t)shift);
            }
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
                           const Limiter& lim, const float* psi, float* G, hipStream_t st) {
    return launch_grad2_t<float>(m, q, a, lim, psi, G, m.geom32, m.recon32, st);
}

hipError_t launch_grad2_64(const snrt_mesh& m, const snrt_quad& q, const StepArgs64& a,
                           const Limiter& lim, const double* psi, double* G, hipStream_t st) {
    return launch_grad2_t<double>(m, q, a, lim, psi, G, m.geom64, m.recon64, st);
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
