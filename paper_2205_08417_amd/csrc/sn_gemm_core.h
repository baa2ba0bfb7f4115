// The block-tile core of the scattering products on the CDNA4 matrix cores (shared by
// the plain products and by the products whose epilogue runs the transport step).
//
// Scattering products C = A X on the CDNA4 matrix cores: the dense kernel S = Psi B of
// eq. SNEqns (B[p][q] = w_p K[q][p], K = N = nq) and the two skinny products of the
// moment-projected form O Sigma M of eq. SNEqns2 (K or N = the padded moment count).
// A is [M][K] FP32 row-major, C is [M][ldc] FP32; K % 32 == 0.  The right operand is stored
// with its N columns zero-padded to a multiple of 128 (the tile width); only the first ldc
// columns of each tile row are written.
//
// Split precision: every FP32 operand x is written as hi + lo with hi = bf16(x) and
// lo = bf16(x - hi) (round to nearest even; x - hi is exact in FP32), and the product is
// accumulated in FP32 as  A_hi B_hi + A_hi B_lo + A_lo B_hi  (the lo*lo term, below 2^-16
// relative, is dropped).  The single-product mode keeps only A_hi B_hi.
//
// FP16 variant (three products, v_mfma_f32_32x32x16_f16): FP16 carries 11 significant bits
// (hi + lo: 22) but only 5 exponent bits, so both operands are scaled by powers of two into
// its range first (exact): every row r of A by 2^e_r with e_r chosen so that the row's largest
// magnitude lands in [2^13, 2^14) (a pre-pass over A writes e_r), and X by one 2^e_B so that
// its largest magnitude lands there too.  The epilogue multiplies each accumulator row by
// 2^-(e_r + e_B), which undoes the scaling exactly.  Entries far below their row's largest
// (below ~2^-16 of it) lose the lo part's precision gradually; their share of a dot product
// is of that order.
//
// Tiling for v_mfma_f32_32x32x16_bf16 (64-lane wavefronts):
//   block tile BM (cells) x BN (ordinates), 8 waves as 2 x 4, each wave BM/2 x BN/4 =
//   BM/64 x BN/128 MFMA tiles with FP32 accumulators.  The main launch uses 256 x 256; the
//   rows of a mostly empty last round of blocks over the compute units go to a second
//   launch with 64 x 128 or 64 x 256 tiles, so that round takes a fraction of the time (the
//   per-element accumulation order, and so the result, does not depend on the tile shape).
//   K runs in chunks of 32 through two LDS stages with one barrier per chunk: after the
//   barrier the block writes chunk k+1 from registers into the idle stage, issues the global
//   loads of chunk k+1+FD into the registers it freed, and multiplies chunk k out of the
//   other stage.  FD = 1 for the full tiles, whose multiply covers the load latency; the
//   small tiles multiply an eighth or a quarter as much per chunk and keep FD = 4 chunks in
//   flight instead.
//   A (Psi, FP32 rows) is split into hi/lo as it is written to LDS; X arrives pre-split
//   and pre-tiled in the LDS plane order (row (kc, n) holds X[kc*32 + kk][n], kk < 32), so
//   one chunk of a block's 256 columns is a contiguous 16 KB run per half, copied to LDS
//   unchanged.  Every LDS plane is [256][32] bf16 (64-byte rows) with the 16-byte granule
//   g of row r stored at position g ^ ((r>>2)&3): the fragment reads of 16 consecutive rows
//   and the stores of 4 consecutive rows then fall on distinct banks without padding.
//   The two waves that share a SIMD run a chunk in different orders (split-then-multiply
//   and half-multiply, split, half-multiply), so one's VALU split overlaps the other's
//   matrix products; without it both split right after the barrier and the matrix core
//   idles (7 % of the product time, measured).
//   Consecutive logical blocks share an A row block (its N tiles) and the XCD-aware block
//   order keeps them on one XCD, so A is fetched from HBM about once.
// MFMA operand layout (32x32x16): lane l supplies row (A) / column (B) l % 32 and the eight
// K values (l / 32) * 8 + [0, 8); accumulator i of lane l is row (i/4)*8 + (l/32)*4 + i%4,
// column l % 32.
#pragma once

#include <algorithm>
#include <type_traits>

#include "snrt_internal.h"

namespace snrt {
namespace gemm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int BK = 32;
constexpr int kThreads = 512;
constexpr int kPlane = 256 * BK;         // bf16 elements of one LDS plane (16 KB)
constexpr int kRsrcWord3 = 0x00020000;

__device__ __forceinline__ uint32_t bf16_rne_bits(float x) {
    uint32_t u = __builtin_bit_cast(uint32_t, x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}

__device__ __forceinline__ float bf16_to_f32(uint32_t h) {
    return __builtin_bit_cast(float, h << 16);
}

// hi/lo split of four floats, packed as four bf16 each (two 32-bit words per half)
__device__ __forceinline__ void split4(f32x4 v, uint32_t (&hi)[2], uint32_t (&lo)[2]) {
    uint32_t h[4], l[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        h[i] = bf16_rne_bits(v[i]);
        l[i] = bf16_rne_bits(v[i] - bf16_to_f32(h[i]));
    }
    hi[0] = h[0] | (h[1] << 16);
    hi[1] = h[2] | (h[3] << 16);
    lo[0] = l[0] | (l[1] << 16);
    lo[1] = l[2] | (l[3] << 16);
}

// FP16 hi/lo split of four floats scaled by 2^e (exact scaling; round to nearest even), packed
// as four halves each (two 32-bit words per half)
__device__ __forceinline__ uint16_t f16_bits(_Float16 h) { return __builtin_bit_cast(uint16_t, h); }

__device__ __forceinline__ void split4_f16(f32x4 v, int e, uint32_t (&hi)[2], uint32_t (&lo)[2]) {
    uint32_t h[4], l[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float x = __builtin_ldexpf(v[i], e);
        const _Float16 xh = (_Float16)x;
        h[i] = f16_bits(xh);
        l[i] = f16_bits((_Float16)(x - (float)xh));
    }
    hi[0] = h[0] | (h[1] << 16);
    hi[1] = h[2] | (h[3] << 16);
    lo[0] = l[0] | (l[1] << 16);
    lo[1] = l[2] | (l[3] << 16);
}

// position of 16-byte granule g in LDS row r
__device__ __forceinline__ int swz(int r, int g) { return g ^ ((r >> 2) & 3); }

// Per-row scalars of the epilogue modes (GemmEpi): kScale a and b, kCombine y in pa.
__device__ __forceinline__ void epi_row(const GemmEpi& epi, int64_t row, float& pa, float& pb) {
    pa = pb = 0.0f;
    if (epi.mode == GemmEpi::kScale) {
        pa = 1.0f + epi.dt * epi.alpha_t * epi.sigma_t[row];
        pb = epi.dt * epi.alpha_s * epi.sigma_s[row];
    } else if (epi.mode == GemmEpi::kCombine) {
        const float cabs = epi.dt * epi.alpha_t * epi.sigma_t[row];
        pa = cabs / (1.0f + cabs);
    }
}

// One accumulated element v through epilogue mode MODE; old is C's previous value (kCombine).
template <int MODE>
__device__ __forceinline__ float epi_val(float v, float old, float pa, float pb, float sg) {
    if constexpr (MODE == GemmEpi::kScale) return v * (pb / (pa - pb * sg));
    if constexpr (MODE == GemmEpi::kCombine) {
        const float x = old + v;
        return x - x * pa;
    }
    return v;
}

// The epilogue of one wave's IM x JN accumulator tiles (32 x 32 each; accumulator r of lane l
// is row row0 + (r/4)*8 + (l/32)*4 + r%4 of the tile, column col0 + l%32).  C is written
// with the streaming bit (read once, by the next kernel or here).  kCombine first loads the
// tile row's previous values, all of them before any store, so the loads overlap.  eu:
// per-row exponents that undo the FP16 scaling (0 otherwise).
template <int MODE, int IM, int JN, typename Acc, typename RowOf, typename ExpOf>
__device__ __forceinline__ void epilogue_tiles(const GemmEpi& epi, Acc (&acc)[IM][JN],
                                               float* __restrict__ C, int64_t M, int32_t ldc,
                                               int col0, int lane, RowOf row_of, ExpOf exp_of) {
#pragma unroll
    for (int i = 0; i < IM; ++i) {
        int eu[16];
        float pa[16], pb[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t row = row_of(i, r);
            eu[r] = exp_of(row);
            pa[r] = pb[r] = 0.0f;
            if constexpr (MODE != GemmEpi::kStore)
                if (row < M) epi_row(epi, row, pa[r], pb[r]);
        }
        float old[JN][16];
#pragma unroll
        for (int j = 0; j < JN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                old[j][r] = 0.0f;
                if constexpr (MODE == GemmEpi::kCombine) {
                    const int col = col0 + j * 32 + (lane & 31);
                    const int64_t row = row_of(i, r);
                    if (col < ldc && row < M) old[j][r] = C[row * ldc + col];
                }
            }
#pragma unroll
        for (int j = 0; j < JN; ++j) {
            const int col = col0 + j * 32 + (lane & 31);
            if (col >= ldc) continue;
            const float sg = MODE == GemmEpi::kScale ? epi.sig[col] : 0.0f;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t row = row_of(i, r);
                const float v = eu[r] != 0 ? __builtin_ldexpf(acc[i][j][r], eu[r]) : acc[i][j][r];
                if (row < M)
                    __builtin_nontemporal_store(epi_val<MODE>(v, old[j][r], pa[r], pb[r], sg),
                                                &C[row * ldc + col]);
            }
        }
    }
}

template <int IM, int JN, typename Acc, typename RowOf, typename ExpOf>
__device__ __forceinline__ void epilogue_any(const GemmEpi& epi, Acc (&acc)[IM][JN],
                                             float* __restrict__ C, int64_t M, int32_t ldc,
                                             int col0, int lane, RowOf row_of, ExpOf exp_of) {
    if (epi.mode == GemmEpi::kScale)
        epilogue_tiles<GemmEpi::kScale>(epi, acc, C, M, ldc, col0, lane, row_of, exp_of);
    else if (epi.mode == GemmEpi::kCombine)
        epilogue_tiles<GemmEpi::kCombine>(epi, acc, C, M, ldc, col0, lane, row_of, exp_of);
    else
        epilogue_tiles<GemmEpi::kStore>(epi, acc, C, M, ldc, col0, lane, row_of, exp_of);
}

// The epilogue's per-row arrays for rows that start at row0 of the full product.
__device__ __forceinline__ GemmEpi epi_rows_from(GemmEpi e, int64_t row0) {
    if (e.sigma_t) e.sigma_t += row0;
    if (e.sigma_s) e.sigma_s += row0;
    return e;
}

// Where a block's accumulator tile sits: rows m0 + wm + ..., columns n0 + wn + ... of the
// product (wm, wn: the wave's origin inside the BM x BN block tile).
struct TileInfo {
    int64_t m0;
    int n0, wm, wn, wave, lane;
};

// One BM x BN block tile of A X; lb is the logical block index (row block major, column
// blocks fastest) and lds the block's two stages of NP planes.  N is the padded width of X
// (a multiple of BN).  F16: FP16 operands with the row exponents rexp[M] of A and the
// exponent eb of X (see the file comment); BF16 otherwise.  The finished accumulators go to
// out(acc, tile, row_of, exp_of): row_of(i, r) is the product row of accumulator r of MFMA
// tile i, exp_of(row) the power of two that undoes the FP16 scaling of that row (0 for BF16).
template <int P, int BM, int BN, int FD, bool STAGGER, bool F16, typename Out>
__device__ __forceinline__ void gemm_block(const float* __restrict__ A,
                                           const uint16_t* __restrict__ Bhi,
                                           const uint16_t* __restrict__ Blo, int64_t M,
                                           int32_t K, int32_t N,
                                           const int32_t* __restrict__ rexp, int32_t eb,
                                           int64_t lb, uint16_t* lds, Out&& out)
{
    using Frag = typename std::conditional<F16, f16x8, bf16x8>::type;
    static_assert(BM == 64 || BM == 128 || BM == 256, "block rows");
    static_assert(BN == 128 || BN == 256, "block columns");
    // P products: A_hi B_hi (+ A_hi B_lo (+ A_lo B_hi)); planes per stage: A hi, B hi, then
    // A lo, B lo (P = 3) or B lo (P = 2)
    static_assert(P >= 1 && P <= 3, "products");
    constexpr int NP = P == 3 ? 4 : P == 2 ? 3 : 2;
    constexpr int PL_AL = 2, PL_BL = P == 3 ? 3 : 2;
    constexpr int IM = BM / 64;          // MFMA tiles per wave along M
    constexpr int JN = BN / 128;         // MFMA tiles per wave along N
    constexpr int AV = BM / 64;          // A float4 per thread per chunk
    constexpr int BV = BN / 128;         // 16-byte B pieces per thread per chunk and half

    const int nN = N / BN;
    const int64_t m0 = (lb / nN) * BM;
    const int n0 = (int)(lb % nN) * BN;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wm = (wave >> 2) * (BM / 2);   // wave tile origin inside the block tile
    const int wn = (wave & 3) * (BN / 4);
    const int nk = K / BK;

    // A rows as a buffer resource: rows past M read as zero
    const uint32_t a_bytes = (uint32_t)((M - m0 < BM ? M - m0 : BM) * (int64_t)K * 4);
    const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(A + m0 * K), 0, (int32_t)a_bytes, kRsrcWord3);

    // global -> register staging of one chunk: A BM x 32 floats = BM * 8 float4 (BM / 64
    // per thread); B BN x 32 bf16 per half = BN * 4 16-byte pieces per half (BN / 128 per
    // thread).  FD register slots hold the chunks kc+1 .. kc+FD, chunk c in slot c % FD.
    f32x4 ga[FD][AV];
    u32x4 gbh[FD][BV], gbl[FD][BV];
    // FP16: the exponent of each A row this thread stages (fixed over the K loop; rows past M
    // read as zero and take exponent 0)
    int ea[AV];
#pragma unroll
    for (int e = 0; e < AV; ++e) {
        const int64_t r = m0 + ((tid + e * kThreads) >> 3);
        ea[e] = (F16 && r < M) ? rexp[r] : 0;
    }
    auto fetch = [&](int kc, int slot) {
#pragma unroll
        for (int e = 0; e < AV; ++e) {
            const int p = tid + e * kThreads;
            const int r = p >> 3, g4 = p & 7;
            i32x4 v = __builtin_amdgcn_raw_buffer_load_b128(
                ra, (uint32_t)((r * K + kc * BK + g4 * 4) * 4), 0, 0);
            ga[slot][e] = __builtin_bit_cast(f32x4, v);
        }
        const size_t tile = ((size_t)kc * N + n0) * BK;
#pragma unroll
        for (int e = 0; e < BV; ++e) {
            const int p = tid + e * kThreads;
            gbh[slot][e] = *reinterpret_cast<const u32x4*>(Bhi + tile + (size_t)p * 8);
            if constexpr (P >= 2)
                gbl[slot][e] = *reinterpret_cast<const u32x4*>(Blo + tile + (size_t)p * 8);
        }
    };
    auto stash = [&](int s, int slot) {
        uint16_t* Ah = lds + (s * NP + 0) * kPlane;
        uint16_t* Bh = lds + (s * NP + 1) * kPlane;
        uint16_t* Al = lds + (s * NP + PL_AL) * kPlane;
        uint16_t* Bl = lds + (s * NP + PL_BL) * kPlane;
#pragma unroll
        for (int e = 0; e < AV; ++e) {
            const int p = tid + e * kThreads;
            const int r = p >> 3, g4 = p & 7;
            const int o = r * BK + swz(r, g4 >> 1) * 8 + (g4 & 1) * 4;
            uint32_t hi[2], lo[2];
            if constexpr (F16)
                split4_f16(ga[slot][e], ea[e], hi, lo);
            else
                split4(ga[slot][e], hi, lo);
            *reinterpret_cast<uint2*>(&Ah[o]) = make_uint2(hi[0], hi[1]);
            if constexpr (P == 3) *reinterpret_cast<uint2*>(&Al[o]) = make_uint2(lo[0], lo[1]);
        }
#pragma unroll
        for (int e = 0; e < BV; ++e) {
            const int p = tid + e * kThreads;    // X is stored in the plane's order
            *reinterpret_cast<u32x4*>(&Bh[p * 8]) = gbh[slot][e];
            if constexpr (P >= 2) *reinterpret_cast<u32x4*>(&Bl[p * 8]) = gbl[slot][e];
        }
    };

    f32x16 acc[IM][JN];
#pragma unroll
    for (int i = 0; i < IM; ++i)
#pragma unroll
        for (int j = 0; j < JN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    const int fr = lane & 31;            // fragment row / column
    // fragment offset inside a plane for K step ks: row fr, granule ks*2 + lane/32 (swizzled;
    // the wave-tile origins are multiples of 32 and leave the swizzle unchanged)
    int foff[2];
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) foff[ks] = fr * BK + swz(fr, ks * 2 + (lane >> 5)) * 8;

    fetch(0, 0);
    stash(0, 0);
#pragma unroll
    for (int d = 1; d <= FD; ++d)
        if (d < nk) fetch(d, d % FD);
    // Waves w and w + 4 share a SIMD.  With STAGGER the second group multiplies the first
    // half of a chunk before staging the next one, so that one wave's hi/lo split (VALU)
    // runs beside the other's matrix products instead of both idling the matrix core
    // right after the barrier.  The products of every accumulator keep their order.
    const bool late = STAGGER && __builtin_amdgcn_readfirstlane(tid >> 8) != 0;

    auto read_frags = [&](int s, int ks, Frag (&ah)[IM], Frag (&al)[IM], Frag (&bh)[JN],
                          Frag (&bl)[JN]) {
        const uint16_t* Ah = lds + (s * NP + 0) * kPlane;
        const uint16_t* Bh = lds + (s * NP + 1) * kPlane;
        const uint16_t* Al = lds + (s * NP + PL_AL) * kPlane;
        const uint16_t* Bl = lds + (s * NP + PL_BL) * kPlane;
#pragma unroll
        for (int j = 0; j < JN; ++j) {
            const int o = (wn + j * 32) * BK + foff[ks];
            bh[j] = *reinterpret_cast<const Frag*>(&Bh[o]);
            if constexpr (P >= 2) bl[j] = *reinterpret_cast<const Frag*>(&Bl[o]);
        }
#pragma unroll
        for (int i = 0; i < IM; ++i) {
            const int o = (wm + i * 32) * BK + foff[ks];
            ah[i] = *reinterpret_cast<const Frag*>(&Ah[o]);
            if constexpr (P == 3) al[i] = *reinterpret_cast<const Frag*>(&Al[o]);
        }
    };
    auto mfma = [](const Frag& a, const Frag& b, const f32x16& c) -> f32x16 {
        if constexpr (F16)
            return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
        else
            return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    };
    auto multiply = [&](const Frag (&ah)[IM], const Frag (&al)[IM], const Frag (&bh)[JN],
                        const Frag (&bl)[JN]) {
#pragma unroll
        for (int i = 0; i < IM; ++i)
#pragma unroll
            for (int j = 0; j < JN; ++j) {
                acc[i][j] = mfma(ah[i], bh[j], acc[i][j]);
                if constexpr (P >= 2) acc[i][j] = mfma(ah[i], bl[j], acc[i][j]);
                if constexpr (P == 3) acc[i][j] = mfma(al[i], bh[j], acc[i][j]);
            }
    };

    // the K loop, unrolled by FD so every register slot index is a constant
    for (int kb = 0; kb < nk; kb += FD) {
#pragma unroll
        for (int u = 0; u < FD; ++u) {
            const int kc = kb + u;
            if (kc >= nk) break;
            const int s = kc & 1;
            __syncthreads();             // chunk kc staged; the idle stage is free again
            auto prepare = [&]() {
                if (kc + 1 < nk) stash(s ^ 1, (u + 1) % FD);
                if (kc + 1 + FD < nk) fetch(kc + 1 + FD, (u + 1) % FD);
            };
            if (!late) prepare();
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                if (late && ks == 1) prepare();
                Frag ah[IM], al[IM], bh[JN], bl[JN];
                read_frags(s, ks, ah, al, bh, bl);
                multiply(ah, al, bh, bl);
            }
        }
    }

    // FP16 rows are scaled back by 2^-(e_r + e_B) on the way out
    auto row_of = [&](int i, int r) -> int64_t {
        return m0 + wm + i * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
    };
    auto exp_of = [&](int64_t row) -> int { return (F16 && row < M) ? -(rexp[row] + eb) : 0; };
    out(acc, TileInfo{m0, n0, wm, wn, wave, lane}, row_of, exp_of);
}


}  // namespace gemm
}  // namespace snrt
