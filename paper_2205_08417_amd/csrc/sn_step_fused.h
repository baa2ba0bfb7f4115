// The explicit dense S_N step in one launch: the scattering product's block tiles run the
// transport update on their own cells and ordinates (kernel templates; instantiated by
// sn_step_fused.hip and sn_step_fused_rho.hip).
//
// The explicit step of Sec. 4.2 with dense scattering (eq. SNEqns) needs the scattering
// source S = Psi B only at the cell and ordinate it updates.  When a block of the product
// finishes its K loop, its accumulators hold S for a tile of cells x ordinates.  Instead of
// writing the tile out for a second kernel to read back, the block stages it in LDS (the K
// loop's operand planes are free by then) and updates those cells and ordinates itself:
// the own row, the neighbour rows, the boundary ghosts and the cell records come from
// memory as in the step kernel, S from LDS, and the new rows go to psi_out.  The update
// arithmetic is the step kernel's own (fwd_load_stage / fwd_compute) on the same operand
// values, so the result equals the two-launch step bit for bit; the S round trip through
// memory (write and read of M x nq floats) disappears.
//
// A tile of 256 cells x 256 ordinates needs 256 KB of FP32 S, twice the LDS the block holds,
// so it runs as two slabs of 256 cells x 128 ordinates: slab s holds, of every wave's two
// 32-column accumulator blocks, block s.  Each wave writes the accumulators of the slab
// (half of its own), then all eight waves update the slab's cells, one cell per wave at a
// time with the step kernel's load pipeline (neighbour lists two cells ahead, rows one cell
// ahead); only half of the accumulators stay live meanwhile.  Lane l owns V = slab width / 64
// consecutive ordinates of the slab; the update is elementwise in the ordinate, so which
// lane owns which ordinate does not change the result.  The LDS rows are stored with their
// 128-byte halves swapped on every other group of 4 rows, so the accumulator writes of the
// two half-waves (rows r and r + 4) fall on different banks.
#pragma once

#include "sn_gemm_core.h"
#include "sn_step_kernels.h"

namespace snrt {
namespace fused {

constexpr int kSlabFloats = 32768;   // 128 KB: the column slabs and the last-round tiles
constexpr bool kRowSlabs = true;     // 256 x 256 tiles as two row slabs (see step_tile)
constexpr int kRowSplit = 160;       // rows of the first row slab
constexpr int kSlabFloatsMax = 40960;  // 160 KB, all the LDS a compute unit has

__device__ __forceinline__ int slab_swz(int row) { return ((row >> 2) & 1) << 5; }

template <int P, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (P < N) {
        f(std::integral_constant<int, P>{});
        static_for<P + 1, N>(f);
    }
}

constexpr int kAhead = 2;            // cells whose rows are in flight ahead of the update

// This wave's accumulators of slab s (tile rows [rs, re)) into the LDS slab sl: column
// slabs hold blocks j = jj * NS + s at slab column (w4 * JS + jj) * 32; row slabs every block
// of the rows they hold.  exp_of undoes the FP16 row scaling.
template <bool RS, int NS, int W, int JS, int IM, int JN, typename Acc, typename ExpOf>
__device__ __forceinline__ void slab_store(Acc (&acc)[IM][JN], const gemm::TileInfo& t, int s,
                                           int rs, int re, ExpOf exp_of,
                                           float* __restrict__ sl) {
    const int lane = t.lane;
    const int w4 = __builtin_amdgcn_readfirstlane(t.wave) & 3;
#pragma unroll
    for (int i = 0; i < IM; ++i) {
        if (RS && (t.wm + i * 32 < rs || t.wm + i * 32 >= re)) continue;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int lr = t.wm + i * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
            const int sr = lr - rs;
            const int e = exp_of(t.m0 + lr);
#pragma unroll
            for (int jj = 0; jj < JS; ++jj) {
                const int j = RS ? jj : jj * NS + s;
                const int lc = (w4 * JS + jj) * 32 + (lane & 31);
                const float v = e != 0 ? __builtin_ldexpf(acc[i][j][r], e) : acc[i][j][r];
                sl[sr * W + (lc ^ slab_swz(sr))] = v;
            }
        }
    }
}

// The update of one block tile: acc holds S for rows m0 + [0, BM) of a sub-product whose
// row 0 is cell row0 (M rows in all), columns n0 + [0, BN); exp_of undoes the FP16 row
// scaling.
template <int BM, int BN, bool RHO, bool DOSE, int D, int IM, int JN, typename Acc,
          typename ExpOf>
__device__ __forceinline__ void step_tile(Acc (&acc)[IM][JN], const gemm::TileInfo& t,
                                          int64_t row0, int64_t M, ExpOf exp_of,
                                          float* __restrict__ sl, const StepEpi& se)
{
    // A tile larger than the LDS slab runs as two slabs: with kRowSlabs, rows [0, kRowSplit)
    // and [kRowSplit, BM) at the full width (V = 4: the rows of 160 cells fill the 160 KB of
    // LDS); otherwise the interleaved column halves described above (V = 2).
    constexpr int NS = BM * BN <= kSlabFloats ? 1 : 2;
    constexpr bool RS = kRowSlabs && NS == 2;
    constexpr int W = RS ? BN : BN / NS;                    // slab width
    constexpr int JS = RS ? JN : JN / NS;                   // accumulator blocks per slab
    constexpr int V = W / 64;                               // ordinates per lane
    static_assert(RS ? kRowSplit * W <= kSlabFloatsMax && kRowSplit % 32 == 0
                     : BM * W <= kSlabFloats && JN % NS == 0, "slab shape");
    static_assert(W >= 64, "slab width");
    constexpr int MF = 3;
    const int lane = t.lane;
    const int wave = __builtin_amdgcn_readfirstlane(t.wave);
    const int64_t trows = M - t.m0 < BM ? M - t.m0 : BM;    // rows of this tile (> 0)

    FwdCtx<float> cx;
    cx.row_bytes = (uint32_t)se.nq * (uint32_t)sizeof(float);
    const uint32_t state_bytes = (uint32_t)se.nc * cx.row_bytes;
    cx.psi = make_rsrc(se.psi_in, state_bytes);
    cx.out = make_rsrc(se.psi_out, state_bytes);
    cx.inflow = make_rsrc(se.a.inflow ? se.a.inflow : se.psi_in,
                          se.a.inflow ? se.nbf * cx.row_bytes : 0u);
    cx.S = make_rsrc(se.psi_in, 0u);                           // S comes from LDS
    cx.src_arr = se.a.source ? se.a.source : se.a.sigma_t;
    cx.src_mul = se.a.source ? se.a.dt : 0.0f;
    cx.inflow_scale = se.a.inflow_scale;
    cx.dirichlet = se.a.inflow != nullptr && !se.a.neumann;
    cx.neumann = se.a.neumann != 0;
    cx.dpart = nullptr;
    const uint32_t cb = (uint32_t)t.n0 * (uint32_t)sizeof(float);
    const int64_t base = row0 + t.m0;

#pragma unroll
    for (int s = 0; s < NS; ++s) {
        // the slab's tile rows [rs, re)
        const int rs = RS && s == 1 ? kRowSplit : 0;
        const int re = RS && s == 0 ? kRowSplit : BM;
        __syncthreads();              // the K loop's planes, or the previous slab, are done
        slab_store<RS, NS, W, JS>(acc, t, s, rs, re, exp_of, sl);
        __syncthreads();
        const int nrow = (trows < re ? (int)trows : re) - rs;   // rows of the slab in M
        if (wave >= nrow) continue;
        // loads run ahead on clamped rows (always in the slab); only rows < nrow are stored
        auto cell = [&](int k) {
            return uniform_cell((int32_t)(base + rs + (k < nrow ? k : nrow - 1)));
        };
        // lane l: slab columns [V l, V l + V), block b = V l / 32 of the slab order, i.e.
        // tile columns (b / JS) * BN/4 + 32 ((b % JS) NS + s) + (V l) % 32 + [0, V)
        const int e0 = lane * V;
        const int blk = e0 >> 5;
        const int q0 = RS ? e0 : (blk / JS) * (BN / 4) + 32 * ((blk % JS) * NS + s) + (e0 & 31);
        float ox[V], oy[V], wi[V];
        load_slice<V, true>(se.tab, t.n0 + q0, se.nq, ox);
        load_slice<V, true>(se.tab + se.nq, t.n0 + q0, se.nq, oy);
#pragma unroll
        for (int k = 0; k < V; ++k) wi[k] = 0.0f;              // unused by the dense update
        // the fused dose: FP64 weights of the lane's ordinates, and the piece of the row this
        // slab (or half-wave, for a 256-wide slab) sums: 128 ordinates each, (n0 / 128) + h
        double wd[DOSE ? V : 1];
        if constexpr (DOSE) {
#pragma unroll
            for (int k = 0; k < V; ++k) wd[k] = se.wq[t.n0 + q0 + k];
        }
        const int npieces = se.nq >> 7;
        const int piece = (t.n0 >> 7) + (W == 256 ? (lane >> 5) : (NS == 2 ? s : 0));
        auto src_of = [&](FwdStage<V, MF, true, float>& d, int k) {
            const float* p = sl + k * W + (e0 ^ slab_swz(k));
#pragma unroll
            for (int v = 0; v < V; ++v) d.src[v] = p[v];
        };
        // The wave's cells of the slab are k = wave + 8 n, n < U <= 32.  Everything a cell's
        // update needs besides its rows (neighbours, normals, ghost scales, coefficients) is
        // loaded up front, cell n in lane n, and read back with readlane: the loop then holds
        // no scalar loads, whose wait would also cover the LDS read of S, and the row loads of
        // a cell depend on no other load.  The rows run D cells ahead of the update, through
        // D + 1 stage slots (cell n in slot n % (D + 1)).  The values are formed exactly as
        // fwd_load_stage forms them.
        const int U = (nrow - wave + 7) / 8;
        int32_t lj[MF];
        float lg[MF], lnx[MF], lny[MF];
        float lirho, lcabs, lcflux, lcscat, lsrcv;
        {
            const int kk = wave + 8 * (lane < 32 ? lane : 31);
            const int32_t c = (int32_t)(base + rs + (kk < nrow ? kk : nrow - 1));
            const CellGeom32* g = se.geom + c;
            lirho = RHO ? se.a.inv_rho[c] : 1.0f;
            const float bscale = cx.dirichlet ? cx.inflow_scale : (cx.neumann ? lirho : 0.0f);
#pragma unroll
            for (int f = 0; f < MF; ++f) {
                const int32_t j = g->nbr[f];
                const bool bnd = j < 0;
                lj[f] = j;
                const float rho_j = RHO ? se.a.inv_rho[bnd ? c : j] : 1.0f;
                lg[f] = bnd ? bscale : rho_j;
                lnx[f] = g->n[f][0];
                lny[f] = g->n[f][1];
            }
            lcabs = se.a.dt * se.a.alpha_t * se.a.sigma_t[c];
            lcflux = se.a.dt * g->inv_area;
            lcscat = se.a.dt * se.a.alpha_s * se.a.sigma_s[c];
            lsrcv = cx.src_arr[c];
        }
        auto rl = [](float v, int l) {
            return __builtin_bit_cast(float,
                                      __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
        };
        FwdStage<V, MF, true, float> st[D + 1];
        // prefetches past the wave's last cell take lane min(n, 31), some cell of the tile:
        // in bounds, and never updated
        auto fetch = [&](auto slot_c, int n) {
            constexpr int SL = decltype(slot_c)::value;
            FwdStage<V, MF, true, float>& d = st[SL];
            const int ln = n < 31 ? n : 31;
            const int32_t c = cell(wave + 8 * n);
            buf_load_row<V, true, float>(cx.psi, (uint32_t)c * cx.row_bytes + cb, q0, se.nq,
                                         d.p);
#pragma unroll
            for (int f = 0; f < MF; ++f) {
                const int32_t j = __builtin_amdgcn_readlane(lj[f], ln);
                const bool bnd = j < 0;
                const int32_t bidx = cx.dirichlet ? -1 - j : c;
                const uint32_t off = (uint32_t)(bnd ? bidx : j) * cx.row_bytes + cb;
                buf_load_row<V, true, float>(bnd && cx.dirichlet ? cx.inflow : cx.psi, off, q0,
                                             se.nq, d.up[f]);
            }
        };
        // the scalars of cell n (n < U) into its slot, just before its update
        auto scalars = [&](FwdStage<V, MF, true, float>& d, int n) {
#pragma unroll
            for (int f = 0; f < MF; ++f) {
                d.ghost[f] = rl(lg[f], n);
                d.nx[f] = rl(lnx[f], n);
                d.ny[f] = rl(lny[f], n);
            }
            d.irho = rl(lirho, n);
            d.cabs = rl(lcabs, n);
            d.cflux = rl(lcflux, n);
            d.cscat = rl(lcscat, n);
            d.srcv = rl(lsrcv, n);
        };
        auto update = [&](auto slot_c, int n) {
            constexpr int SL = decltype(slot_c)::value;
            const int k = wave + 8 * n;
            scalars(st[SL], n);
            src_of(st[SL], k);
            fwd_compute<V, true, MF, RHO, true, float>(st[SL], ox, oy, wi, cell(k), cb, se.nq,
                                                       q0, cx);
            if constexpr (DOSE) {
                double sd = 0.0;
#pragma unroll
                for (int v = 0; v < V; ++v) sd += wd[v] * (double)st[SL].p[v];
                // sum over the lanes of the piece: the whole wave, or each half of it
#pragma unroll
                for (int off = (W == 256 ? 16 : 32); off >= 1; off >>= 1)
                    sd += __shfl_xor(sd, off, kWave);
                if ((lane & (W == 256 ? 31 : 63)) == 0)
                    se.dpart[(int64_t)cell(k) * npieces + piece] = sd;
            }
        };
        static_for<0, D>([&](auto d_c) { fetch(d_c, decltype(d_c)::value); });
        for (int n = 0; n < U; n += D + 1) {
            static_for<0, D + 1>([&](auto p_c) {
                constexpr int P = decltype(p_c)::value;
                if (n + P < U) {
                    fetch(std::integral_constant<int, (P + D) % (D + 1)>{}, n + P + D);
                    update(p_c, n + P);
                }
            });
        }
    }
}

// Blocks [0, nmain) are 256 x 256 tiles of the first M1 rows, blocks [nmain, grid) TM x TN
// tiles of the rest (the block order and last-round policy of the plain product).
template <bool F16, int P, int TM, int TN, bool STAGGER, bool RHO, bool DOSE>
__global__ __launch_bounds__(gemm::kThreads) void k_gemm_step(
    const float* __restrict__ A, const uint16_t* __restrict__ Bhi,
    const uint16_t* __restrict__ Blo, int64_t M1, int64_t M, int32_t K, int32_t N,
    const int32_t* __restrict__ rexp, int32_t eb, int64_t nmain, StepEpi se)
{
    constexpr int NP = P == 3 ? 4 : P == 2 ? 3 : 2;
    constexpr int kPlanes = 2 * NP * gemm::kPlane;
    constexpr int kSlab = kRowSlabs ? kRowSplit * 256 : kSlabFloats;
    constexpr int kU16 = kPlanes > 2 * kSlab ? kPlanes : 2 * kSlab;
    __shared__ __attribute__((aligned(16))) uint16_t lds[kU16];
    float* sl = reinterpret_cast<float*>(lds);
    const int64_t b = blockIdx.x;
    if (b < nmain) {
        gemm::gemm_block<P, 256, 256, 1, STAGGER, F16>(
            A, Bhi, Blo, M1, K, N, rexp, eb, xcd_remap(b, nmain), lds,
            [&](auto& acc, const gemm::TileInfo& t, auto, auto exp_of) {
                step_tile<256, 256, RHO, DOSE, kAhead>(acc, t, 0, M1, exp_of, sl, se);
            });
    } else {
        const int64_t nt = (int64_t)gridDim.x - nmain;
        gemm::gemm_block<P, TM, TN, 4, STAGGER, F16>(
            A + M1 * K, Bhi, Blo, M - M1, K, N, F16 ? rexp + M1 : rexp, eb,
            xcd_remap(b - nmain, nt), lds,
            [&](auto& acc, const gemm::TileInfo& t, auto, auto exp_of) {
                step_tile<TM, TN, RHO, DOSE, kAhead>(acc, t, M1, M - M1, exp_of, sl, se);
            });
    }
}

template <bool RHO, bool DOSE>
hipError_t launch_gemm_step_t(const float* A, const uint16_t* Bhi, const uint16_t* Blo,
                              int64_t M, int32_t K, int32_t N, int products,
                              const int32_t* rexp, int32_t eb, const StepEpi& se,
                              hipStream_t st)
{
    if (M == 0) return hipSuccess;
    if (products < 0 || products > 3) return hipErrorInvalidValue;
    if (K % 32 != 0 || K == 0 || N % 256 != 0 || N != se.nq || M != se.nc ||
        (products == 0 && !rexp) || RHO != (se.a.inv_rho != nullptr) ||
        DOSE != (se.dpart != nullptr) || (DOSE && !se.wq))
        return hipErrorNotSupported;
    const GemmPlan p = gemm_plan(M, N);
    if (p.mbn != 256) return hipErrorNotSupported;
    const int64_t nmain = ((p.rows1 + 255) / 256) * (N / 256);
    const int64_t ntail = ((M - p.rows1 + p.tm - 1) / p.tm) * (N / p.tn);
    const dim3 grid((unsigned)(nmain + ntail));
    const bool stagger = tune().gemm_stagger && K >= 256 && N >= 256;
    auto go = [&](auto p_c, auto tn_c, auto sg_c) {
        constexpr int PP = decltype(p_c)::value;
        constexpr int TN = decltype(tn_c)::value;
        constexpr bool SG = decltype(sg_c)::value;
        hipLaunchKernelGGL((k_gemm_step<PP == 0, PP == 0 ? 3 : PP, 64, TN, SG, RHO, DOSE>), grid,
                           dim3(gemm::kThreads), 0, st, A, Bhi, Blo, p.rows1, M, K, N, rexp, eb,
                           nmain, se);
        return hipGetLastError();
    };
    auto by_tn = [&](auto p_c, auto sg_c) {
        return p.tn == 128 ? go(p_c, std::integral_constant<int, 128>{}, sg_c)
                           : go(p_c, std::integral_constant<int, 256>{}, sg_c);
    };
    auto by_sg = [&](auto p_c) {
        return stagger ? by_tn(p_c, std::true_type{}) : by_tn(p_c, std::false_type{});
    };
    switch (products) {
        case 0: return by_sg(std::integral_constant<int, 0>{});
        case 3: return by_sg(std::integral_constant<int, 3>{});
        case 2: return by_sg(std::integral_constant<int, 2>{});
        default: return by_sg(std::integral_constant<int, 1>{});
    }
}

// The last factor of the mode-space IMEX solve (IMEX step of Sec. 4.2) in the same tile
// form: acc holds S for its cells and ordinates, out holds the collision-free step r, and
// each element becomes x - x y with x = r + S and y = c / (1 + c), c = dt alpha_t sigma_t of
// the cell (the kCombine epilogue's arithmetic), written over r.  Rows run at full width
// through the row slabs with V = 4 ordinates per lane; y of the wave's cells sits in lanes.
template <int BM, int BN, int D, int IM, int JN, typename Acc, typename ExpOf>
__device__ __forceinline__ void combine_tile(Acc (&acc)[IM][JN], const gemm::TileInfo& t,
                                             int64_t row0, int64_t M, ExpOf exp_of,
                                             float* __restrict__ sl, const CombineEpi& ce)
{
    constexpr int NS = BM * BN <= kSlabFloats ? 1 : 2;
    static_assert(kRowSlabs || NS == 1, "the combine runs on row slabs");
    constexpr bool RS = NS == 2;
    constexpr int W = BN, V = W / 64;
    const int lane = t.lane;
    const int wave = __builtin_amdgcn_readfirstlane(t.wave);
    const int64_t trows = M - t.m0 < BM ? M - t.m0 : BM;
    const uint32_t row_bytes = (uint32_t)ce.nq * (uint32_t)sizeof(float);
    const __amdgpu_buffer_rsrc_t out = make_rsrc(ce.out, (uint32_t)ce.nc * row_bytes);
    const uint32_t cb = (uint32_t)t.n0 * (uint32_t)sizeof(float);
    const int64_t base = row0 + t.m0;
    const int q0 = lane * V;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int rs = RS && s == 1 ? kRowSplit : 0;
        const int re = RS && s == 0 ? kRowSplit : BM;
        __syncthreads();
        slab_store<RS, NS, W, JN>(acc, t, s, rs, re, exp_of, sl);
        __syncthreads();
        const int nrow = (trows < re ? (int)trows : re) - rs;
        if (wave >= nrow) continue;
        auto cell = [&](int k) {
            return uniform_cell((int32_t)(base + rs + (k < nrow ? k : nrow - 1)));
        };
        const int U = (nrow - wave + 7) / 8;                    // <= kRowSplit / 8 <= 32
        float ly;                                               // y of the wave's cell n
        {
            const int kk = wave + 8 * (lane < 32 ? lane : 31);
            const int32_t c = (int32_t)(base + rs + (kk < nrow ? kk : nrow - 1));
            const float cabs = ce.dt * ce.alpha_t * ce.sigma_t[c];
            ly = cabs / (1.0f + cabs);
        }
        float st[D + 1][V];
        auto fetch = [&](auto slot_c, int n) {
            constexpr int SL = decltype(slot_c)::value;
            buf_load_row<V, true, float>(out, (uint32_t)cell(wave + 8 * n) * row_bytes + cb, q0,
                                         ce.nq, st[SL]);
        };
        auto update = [&](auto slot_c, int n) {
            constexpr int SL = decltype(slot_c)::value;
            const int k = wave + 8 * n;
            const float y = __builtin_bit_cast(
                float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, ly), n));
            const float* p = sl + k * W + (q0 ^ slab_swz(k));
            float o[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const float x = st[SL][v] + p[v];
                o[v] = __builtin_fmaf(-x, y, x);
            }
            buf_store_row<V, true, float, kAuxStream>(out, (uint32_t)cell(k) * row_bytes + cb,
                                                      q0, ce.nq, o);
        };
        static_for<0, D>([&](auto d_c) { fetch(d_c, decltype(d_c)::value); });
        for (int n = 0; n < U; n += D + 1) {
            static_for<0, D + 1>([&](auto p_c) {
                constexpr int P = decltype(p_c)::value;
                if (n + P < U) {
                    fetch(std::integral_constant<int, (P + D) % (D + 1)>{}, n + P + D);
                    update(p_c, n + P);
                }
            });
        }
    }
}

template <bool F16, int P, int TM, int TN, bool STAGGER>
__global__ __launch_bounds__(gemm::kThreads) void k_gemm_combine(
    const float* __restrict__ A, const uint16_t* __restrict__ Bhi,
    const uint16_t* __restrict__ Blo, int64_t M1, int64_t M, int32_t K, int32_t N,
    const int32_t* __restrict__ rexp, int32_t eb, int64_t nmain, CombineEpi ce)
{
    constexpr int NP = P == 3 ? 4 : P == 2 ? 3 : 2;
    constexpr int kPlanes = 2 * NP * gemm::kPlane;
    constexpr int kSlab = kRowSlabs ? kRowSplit * 256 : kSlabFloats;
    constexpr int kU16 = kPlanes > 2 * kSlab ? kPlanes : 2 * kSlab;
    __shared__ __attribute__((aligned(16))) uint16_t lds[kU16];
    float* sl = reinterpret_cast<float*>(lds);
    const int64_t b = blockIdx.x;
    if (b < nmain) {
        gemm::gemm_block<P, 256, 256, 1, STAGGER, F16>(
            A, Bhi, Blo, M1, K, N, rexp, eb, xcd_remap(b, nmain), lds,
            [&](auto& acc, const gemm::TileInfo& t, auto, auto exp_of) {
                combine_tile<256, 256, kAhead>(acc, t, 0, M1, exp_of, sl, ce);
            });
    } else {
        const int64_t nt = (int64_t)gridDim.x - nmain;
        gemm::gemm_block<P, TM, TN, 4, STAGGER, F16>(
            A + M1 * K, Bhi, Blo, M - M1, K, N, F16 ? rexp + M1 : rexp, eb,
            xcd_remap(b - nmain, nt), lds,
            [&](auto& acc, const gemm::TileInfo& t, auto, auto exp_of) {
                combine_tile<TM, TN, kAhead>(acc, t, M1, M - M1, exp_of, sl, ce);
            });
    }
}


// The transposed dense step of one block tile (the last transposed product's S holds
// G = Lambda B^T for its cells and ordinates): the arithmetic of adj_compute for dense
// scattering (adj_downwind_sum, adj_update, explicit FMAs), rows at full width through the
// row slabs, four ordinates per lane; the cell data of the wave's cells in lanes.  DA: the
// dose functional's term on the output rows.
template <int BM, int BN, bool DA, int D, int IM, int JN, typename Acc, typename ExpOf>
__device__ __forceinline__ void adjoint_tile(Acc (&acc)[IM][JN], const gemm::TileInfo& t,
                                             int64_t row0, int64_t M, ExpOf exp_of,
                                             float* __restrict__ sl, const AdjEpi& ae)
{
    constexpr int NS = BM * BN <= kSlabFloats ? 1 : 2;
    static_assert(kRowSlabs || NS == 1, "the transposed step runs on row slabs");
    constexpr bool RS = NS == 2;
    constexpr int W = BN, V = W / 64;
    constexpr int MF = 3;
    using Stage = AdjStage<V, MF, true, float, double>;
    const int lane = t.lane;
    const int wave = __builtin_amdgcn_readfirstlane(t.wave);
    const int64_t trows = M - t.m0 < BM ? M - t.m0 : BM;
    const uint32_t row_bytes = (uint32_t)ae.nq * (uint32_t)sizeof(float);
    const uint32_t state_bytes = (uint32_t)ae.nc * row_bytes;
    const auto rlam = make_rsrc(ae.lam_np1, state_bytes);
    const auto rpsi = make_rsrc(ae.psi_n, state_bytes);
    const auto rout = make_rsrc(ae.lam_n, state_bytes);
    const uint32_t cb = (uint32_t)t.n0 * (uint32_t)sizeof(float);
    const int64_t base = row0 + t.m0;
    const int q0 = lane * V;
    const StepArgs32& a = ae.a;
    const bool neumann = a.neumann != 0;
    float ox[V], oy[V];
    load_slice<V, true>(ae.tab, t.n0 + q0, ae.nq, ox);
    load_slice<V, true>(ae.tab + ae.nq, t.n0 + q0, ae.nq, oy);
    double wd[DA ? V : 1];
    if constexpr (DA) load_slice<V, true>(ae.da.w, t.n0 + q0, ae.nq, wd);
    const int npieces = ae.nq >> 7;
    const int piece = (t.n0 >> 7) + (W == 256 ? (lane >> 5) : 0);
    auto rl = [](float v, int l) {
        return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
    };
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int rs = RS && s == 1 ? kRowSplit : 0;
        const int re = RS && s == 0 ? kRowSplit : BM;
        __syncthreads();
        slab_store<RS, NS, W, JN>(acc, t, s, rs, re, exp_of, sl);
        __syncthreads();
        const int nrow = (trows < re ? (int)trows : re) - rs;
        if (wave >= nrow) continue;
        auto cell = [&](int k) {
            return uniform_cell((int32_t)(base + rs + (k < nrow ? k : nrow - 1)));
        };
        const int U = (nrow - wave + 7) / 8;                    // <= 32
        // cell data of the wave's cell n in lane n, formed as adj_load_stage forms it
        int32_t lsrc[MF];
        float lian[MF], lnx[MF], lny[MF];
        int lsign = 0;
        float lia, lirho, lcabs, lcscat;
        double lgd = 0.0;
        {
            const int kk = wave + 8 * (lane < 32 ? lane : 31);
            const int32_t c = (int32_t)(base + rs + (kk < nrow ? kk : nrow - 1));
            const CellGeom32* g = ae.geom + c;
#pragma unroll
            for (int f = 0; f < MF; ++f) {
                const int32_t j = g->nbr[f];
                const bool interior = j >= 0;
                const int32_t src = interior ? j : c;
                lsrc[f] = src;
                lian[f] = interior ? ae.geom[src].inv_area : 0.0f;
                lsign |= (!interior && neumann) ? (1 << f) : 0;
                lnx[f] = g->n[f][0];
                lny[f] = g->n[f][1];
            }
            lia = g->inv_area;
            lirho = a.inv_rho ? a.inv_rho[c] : 1.0f;
            lcabs = a.dt * a.alpha_t * a.sigma_t[c];
            lcscat = a.dt * a.alpha_s * a.sigma_s[c];
            if constexpr (DA)
                lgd = ae.da.coeff * (a.inv_rho ? (double)a.inv_rho[c] : 1.0) * ae.da.g_dose[c];
        }
        Stage st[D + 1];
        auto fetch = [&](auto slot_c, int n) {
            constexpr int SL = decltype(slot_c)::value;
            Stage& d = st[SL];
            const int ln = n < 31 ? n : 31;
            const uint32_t own = (uint32_t)cell(wave + 8 * n) * row_bytes + cb;
            buf_load_row<V, true, float>(rlam, own, q0, ae.nq, d.l);
            buf_load_row<V, true, float>(rpsi, own, q0, ae.nq, d.p);
#pragma unroll
            for (int f = 0; f < MF; ++f) {
                const int32_t src = __builtin_amdgcn_readlane(lsrc[f], ln);
                buf_load_row<V, true, float>(rlam, (uint32_t)src * row_bytes + cb, q0, ae.nq,
                                             d.ln[f]);
            }
        };
        auto update = [&](auto slot_c, int n) {
            constexpr int SL = decltype(slot_c)::value;
            Stage& d = st[SL];
            const int k = wave + 8 * n;
            const int sg = __builtin_amdgcn_readlane(lsign, n);
#pragma unroll
            for (int f = 0; f < MF; ++f) {
                d.ia_n[f] = rl(lian[f], n);
                d.nx[f] = rl(lnx[f], n);
                d.ny[f] = rl(lny[f], n);
                d.all_signs[f] = (sg >> f) & 1;
            }
            d.ia = rl(lia, n);
            const float irho = rl(lirho, n);
            const float cabs = rl(lcabs, n);
            const float cscat = rl(lcscat, n);
            const float* p = sl + k * W + (q0 ^ slab_swz(k));
            float g[V];
#pragma unroll
            for (int v = 0; v < V; ++v) g[v] = p[v];
            float xs[V];
#pragma unroll
            for (int v = 0; v < V; ++v) xs[v] = 0.0f;
            adj_downwind_sum(d, ox, oy, xs);
            const float cstream = a.dt * irho;
            float o[V];
            adj_update(d.l, xs, g, cabs, cstream, cscat, o);
            float pt = 0.0f, ps = 0.0f, pr = 0.0f;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                pt = __builtin_fmaf(d.l[v], d.p[v], pt);
                ps = __builtin_fmaf(d.p[v], g[v], ps);
                pr = __builtin_fmaf(d.p[v], xs[v], pr);
            }
            if constexpr (DA) {
                const double gd = __builtin_bit_cast(
                    double, ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(
                                 (int)(__builtin_bit_cast(uint64_t, lgd) >> 32), n) << 32) |
                                (uint64_t)(uint32_t)__builtin_amdgcn_readlane(
                                    (int)(uint32_t)__builtin_bit_cast(uint64_t, lgd), n));
#pragma unroll
                for (int v = 0; v < V; ++v) o[v] = (float)__builtin_fma(gd, wd[v], (double)o[v]);
            }
            const int32_t c = cell(k);
            buf_store_row<V, true, float, kAuxStream>(rout, (uint32_t)c * row_bytes + cb, q0,
                                                      ae.nq, o);
            // the piece's gradient sums: the whole wave, or each half of it
#pragma unroll
            for (int off = (W == 256 ? 16 : 32); off >= 1; off >>= 1) {
                pt += __shfl_xor(pt, off, kWave);
                ps += __shfl_xor(ps, off, kWave);
                pr += __shfl_xor(pr, off, kWave);
            }
            if ((lane & (W == 256 ? 31 : 63)) == 0) {
                float* q = ae.part + ((int64_t)c * npieces + piece) * 3;
                q[0] = pt;
                q[1] = ps;
                q[2] = pr;
            }
        };
        static_for<0, D>([&](auto d_c) { fetch(d_c, decltype(d_c)::value); });
        for (int n = 0; n < U; n += D + 1) {
            static_for<0, D + 1>([&](auto p_c) {
                constexpr int P = decltype(p_c)::value;
                if (n + P < U) {
                    fetch(std::integral_constant<int, (P + D) % (D + 1)>{}, n + P + D);
                    update(p_c, n + P);
                }
            });
        }
    }
}

template <bool F16, int P, int TM, int TN, bool STAGGER, bool DA>
__global__ __launch_bounds__(gemm::kThreads) void k_gemm_adjoint(
    const float* __restrict__ A, const uint16_t* __restrict__ Bhi,
    const uint16_t* __restrict__ Blo, int64_t M1, int64_t M, int32_t K, int32_t N,
    const int32_t* __restrict__ rexp, int32_t eb, int64_t nmain, AdjEpi ae)
{
    constexpr int NP = P == 3 ? 4 : P == 2 ? 3 : 2;
    constexpr int kPlanes = 2 * NP * gemm::kPlane;
    constexpr int kSlab = kRowSlabs ? kRowSplit * 256 : kSlabFloats;
    constexpr int kU16 = kPlanes > 2 * kSlab ? kPlanes : 2 * kSlab;
    __shared__ __attribute__((aligned(16))) uint16_t lds[kU16];
    float* sl = reinterpret_cast<float*>(lds);
    const int64_t b = blockIdx.x;
    if (b < nmain) {
        gemm::gemm_block<P, 256, 256, 1, STAGGER, F16>(
            A, Bhi, Blo, M1, K, N, rexp, eb, xcd_remap(b, nmain), lds,
            [&](auto& acc, const gemm::TileInfo& t, auto, auto exp_of) {
                adjoint_tile<256, 256, DA, kAhead>(acc, t, 0, M1, exp_of, sl, ae);
            });
    } else {
        const int64_t nt = (int64_t)gridDim.x - nmain;
        gemm::gemm_block<P, TM, TN, 4, STAGGER, F16>(
            A + M1 * K, Bhi, Blo, M - M1, K, N, F16 ? rexp + M1 : rexp, eb,
            xcd_remap(b - nmain, nt), lds,
            [&](auto& acc, const gemm::TileInfo& t, auto, auto exp_of) {
                adjoint_tile<TM, TN, DA, kAhead>(acc, t, M1, M - M1, exp_of, sl, ae);
            });
    }
}

template <bool DA>
hipError_t launch_gemm_adjoint_impl(const float* A, const uint16_t* Bhi, const uint16_t* Blo,
                                    int64_t M, int32_t K, int32_t N, int products,
                                    const int32_t* rexp, int32_t eb, const AdjEpi& ae,
                                    hipStream_t st)
{
    if (M == 0) return hipSuccess;
    if (products < 0 || products > 3) return hipErrorInvalidValue;
    if (K % 32 != 0 || K == 0 || N % 256 != 0 || N != ae.nq || M != ae.nc || !ae.part ||
        (products == 0 && !rexp) || (DA && (!ae.da.w || !ae.da.g_dose)))
        return hipErrorNotSupported;
    const GemmPlan p = gemm_plan(M, N);
    if (p.mbn != 256) return hipErrorNotSupported;
    const int64_t nmain = ((p.rows1 + 255) / 256) * (N / 256);
    const int64_t ntail = ((M - p.rows1 + p.tm - 1) / p.tm) * (N / p.tn);
    const dim3 grid((unsigned)(nmain + ntail));
    const bool stagger = tune().gemm_stagger && K >= 256 && N >= 256;
    auto go = [&](auto p_c, auto tn_c, auto sg_c) {
        constexpr int PP = decltype(p_c)::value;
        constexpr int TN = decltype(tn_c)::value;
        constexpr bool SG = decltype(sg_c)::value;
        hipLaunchKernelGGL((k_gemm_adjoint<PP == 0, PP == 0 ? 3 : PP, 64, TN, SG, DA>), grid,
                           dim3(gemm::kThreads), 0, st, A, Bhi, Blo, p.rows1, M, K, N, rexp, eb,
                           nmain, ae);
        return hipGetLastError();
    };
    auto by_tn = [&](auto p_c, auto sg_c) {
        return p.tn == 128 ? go(p_c, std::integral_constant<int, 128>{}, sg_c)
                           : go(p_c, std::integral_constant<int, 256>{}, sg_c);
    };
    auto by_sg = [&](auto p_c) {
        return stagger ? by_tn(p_c, std::true_type{}) : by_tn(p_c, std::false_type{});
    };
    switch (products) {
        case 0: return by_sg(std::integral_constant<int, 0>{});
        case 3: return by_sg(std::integral_constant<int, 3>{});
        case 2: return by_sg(std::integral_constant<int, 2>{});
        default: return by_sg(std::integral_constant<int, 1>{});
    }
}

}  // namespace fused
}  // namespace snrt
