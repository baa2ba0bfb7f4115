// Scattering products C = A X on the CDNA4 matrix cores: the dense kernel S = Psi B of
// eq. SNEqns (B[p][q] = w_p K[q][p], K = N = nq) and the two skinny products of the
// moment-projected form O Sigma M of eq. SNEqns2 (K or N = the padded moment count).
// A is [M][K] FP32 row-major, C is [M][N] FP32; K % 32 == 0 and N % 256 == 0.
//
// Split precision: every FP32 operand x is written as hi + lo with hi = bf16(x) and
// lo = bf16(x - hi) (round to nearest even; x - hi is exact in FP32), and the product is
// accumulated in FP32 as  A_hi B_hi + A_hi B_lo + A_lo B_hi  (the lo*lo term, below 2^-16
// relative, is dropped).  The single-product mode keeps only A_hi B_hi.
//
// Tiling for v_mfma_f32_32x32x16_bf16 (64-lane wavefronts):
//   block tile 256 (cells) x 256 (ordinates), 8 waves as 2 x 4, each wave 128 x 64 =
//   4 x 2 MFMA tiles with FP32 accumulators.  K runs in chunks of 32 through two LDS
//   stages with one barrier per chunk: after the barrier the block writes chunk k+1 into
//   the idle stage, issues the global loads of chunk k+2 into registers, and multiplies
//   chunk k out of the other stage.
//   A (Psi, FP32 rows) is split into hi/lo as it is written to LDS; X arrives pre-split
//   and pre-tiled (plane[kc][n][kk] = part of X[kc*32 + kk][n]), so one chunk of a block's
//   256 columns is a contiguous 16 KB run per half.  Every LDS plane is [256][32] bf16
//   (64-byte rows) with the 16-byte granule g of row r stored at position g ^ ((r>>2)&3):
//   the fragment reads of 16 consecutive rows and the stores of 4 consecutive rows then
//   fall on distinct banks without padding.
//   Consecutive logical blocks share an A row block (its N tiles) and the XCD-aware block
//   order keeps them on one XCD, so A is fetched from HBM about once.
// MFMA operand layout (32x32x16): lane l supplies row (A) / column (B) l % 32 and the eight
// K values (l / 32) * 8 + [0, 8); accumulator i of lane l is row (i/4)*8 + (l/32)*4 + i%4,
// column l % 32.
#include "snrt_internal.h"

namespace snrt {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = 256, BN = 256, BK = 32;
constexpr int kThreads = 512;
constexpr int kPlane = BM * BK;          // bf16 elements of one LDS plane (16 KB)
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

// position of 16-byte granule g in LDS row r
__device__ __forceinline__ int swz(int r, int g) { return g ^ ((r >> 2) & 3); }

template <bool THREE>
__global__ __launch_bounds__(kThreads) void k_gemm_bf16(const float* __restrict__ A,
                                                        const uint16_t* __restrict__ Bhi,
                                                        const uint16_t* __restrict__ Blo,
                                                        float* __restrict__ C, int64_t M,
                                                        int32_t K, int32_t N)
{
    constexpr int NP = THREE ? 4 : 2;    // planes per stage: A hi, B hi (, A lo, B lo)
    __shared__ __attribute__((aligned(16))) uint16_t lds[2 * NP * kPlane];

    const int nN = N / BN;
    const int64_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t m0 = (lb / nN) * BM;
    const int n0 = (int)(lb % nN) * BN;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wm = (wave >> 2) * 128;    // wave tile origin inside the block tile
    const int wn = (wave & 3) * 64;
    const int nk = K / BK;

    // A rows as a buffer resource: rows past M read as zero
    const uint32_t a_bytes = (uint32_t)((M - m0 < BM ? M - m0 : BM) * (int64_t)K * 4);
    const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(A + m0 * K), 0, (int32_t)a_bytes, kRsrcWord3);

    // global -> register staging of one chunk: A 256 x 32 floats = 2048 float4 (4 per
    // thread); B 256 x 32 bf16 per half = 1024 16-byte pieces per half (2 per thread)
    f32x4 ga[4];
    u32x4 gbh[2], gbl[2];
    auto fetch = [&](int kc) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int p = tid + e * kThreads;
            const int r = p >> 3, g4 = p & 7;
            i32x4 v = __builtin_amdgcn_raw_buffer_load_b128(
                ra, (uint32_t)((r * K + kc * BK + g4 * 4) * 4), 0, 0);
            ga[e] = __builtin_bit_cast(f32x4, v);
        }
        const size_t tile = ((size_t)kc * N + n0) * BK;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int p = tid + e * kThreads;
            gbh[e] = *reinterpret_cast<const u32x4*>(Bhi + tile + (size_t)p * 8);
            if constexpr (THREE) gbl[e] = *reinterpret_cast<const u32x4*>(Blo + tile + (size_t)p * 8);
        }
    };
    auto stash = [&](int s) {
        uint16_t* Ah = lds + (s * NP + 0) * kPlane;
        uint16_t* Bh = lds + (s * NP + 1) * kPlane;
        uint16_t* Al = lds + (s * NP + 2) * kPlane;
        uint16_t* Bl = lds + (s * NP + 3) * kPlane;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int p = tid + e * kThreads;
            const int r = p >> 3, g4 = p & 7;
            const int o = r * BK + swz(r, g4 >> 1) * 8 + (g4 & 1) * 4;
            uint32_t hi[2], lo[2];
            split4(ga[e], hi, lo);
            *reinterpret_cast<uint2*>(&Ah[o]) = make_uint2(hi[0], hi[1]);
            if constexpr (THREE) *reinterpret_cast<uint2*>(&Al[o]) = make_uint2(lo[0], lo[1]);
        }
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int p = tid + e * kThreads;
            const int n = p >> 2, g = p & 3;
            const int o = n * BK + swz(n, g) * 8;
            *reinterpret_cast<u32x4*>(&Bh[o]) = gbh[e];
            if constexpr (THREE) *reinterpret_cast<u32x4*>(&Bl[o]) = gbl[e];
        }
    };

    f32x16 acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    const int fr = lane & 31;            // fragment row / column
    // fragment offset inside a plane for K step ks: row fr, granule ks*2 + lane/32 (swizzled;
    // the wave-tile origins are multiples of 32 and leave the swizzle unchanged)
    int foff[2];
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) foff[ks] = fr * BK + swz(fr, ks * 2 + (lane >> 5)) * 8;

    fetch(0);
    stash(0);
    if (nk > 1) fetch(1);
    for (int kc = 0; kc < nk; ++kc) {
        __syncthreads();                 // chunk kc staged; the idle stage is free again
        const int s = kc & 1;
        if (kc + 1 < nk) stash(s ^ 1);
        if (kc + 2 < nk) fetch(kc + 2);
        const uint16_t* Ah = lds + (s * NP + 0) * kPlane;
        const uint16_t* Bh = lds + (s * NP + 1) * kPlane;
        const uint16_t* Al = lds + (s * NP + 2) * kPlane;
        const uint16_t* Bl = lds + (s * NP + 3) * kPlane;
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            bf16x8 ah[4], al[4], bh[2], bl[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int o = (wn + j * 32) * BK + foff[ks];
                bh[j] = *reinterpret_cast<const bf16x8*>(&Bh[o]);
                if constexpr (THREE) bl[j] = *reinterpret_cast<const bf16x8*>(&Bl[o]);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int o = (wm + i * 32) * BK + foff[ks];
                ah[i] = *reinterpret_cast<const bf16x8*>(&Ah[o]);
                if constexpr (THREE) al[i] = *reinterpret_cast<const bf16x8*>(&Al[o]);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
                    if constexpr (THREE) {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                    }
                }
        }
    }

    // epilogue: accumulator r of lane l is row (r/4)*8 + (l/32)*4 + r%4, column l%32; S is
    // consumed once by the step kernel, so it is streamed past the caches
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int col = n0 + wn + j * 32 + fr;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t row = m0 + wm + i * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
                if (row < M) __builtin_nontemporal_store(acc[i][j][r], &C[row * N + col]);
            }
        }
}

// Tiled halves of X [K][N]: hi[(kc*N + n)*32 + kk] = bf16(X[kc*32 + kk][n]), lo = bf16(X - hi)
__global__ __launch_bounds__(256) void k_split(const float* __restrict__ B, uint16_t* __restrict__ hi,
                                               uint16_t* __restrict__ lo, int32_t K, int32_t N)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)K * N) return;
    const int kk = (int)(i % BK);
    const int64_t t = i / BK;
    const int n = (int)(t % N);
    const int kc = (int)(t / N);
    const float x = B[(int64_t)(kc * BK + kk) * N + n];
    const uint32_t h = bf16_rne_bits(x);
    hi[i] = (uint16_t)h;
    lo[i] = (uint16_t)bf16_rne_bits(x - bf16_to_f32(h));
}

}  // namespace

hipError_t launch_split_bf16(const float* B, uint16_t* hi, uint16_t* lo, int32_t K, int32_t N,
                             hipStream_t st) {
    if (K % BK != 0 || N % BN != 0) return hipErrorNotSupported;
    const int64_t n = (int64_t)K * N;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_split, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, B, hi, lo, K, N);
    return hipGetLastError();
}

hipError_t launch_gemm_bf16(const float* A, const uint16_t* Bhi, const uint16_t* Blo, float* C,
                            int64_t M, int32_t K, int32_t N, bool three_products, hipStream_t st) {
    if (M == 0) return hipSuccess;
    if (K % BK != 0 || N % BN != 0 || K == 0) return hipErrorNotSupported;
    const int64_t blocks = ((M + BM - 1) / BM) * (N / BN);
    if (three_products)
        hipLaunchKernelGGL(k_gemm_bf16<true>, dim3((unsigned)blocks), dim3(kThreads), 0, st, A,
                           Bhi, Blo, C, M, K, N);
    else
        hipLaunchKernelGGL(k_gemm_bf16<false>, dim3((unsigned)blocks), dim3(kThreads), 0, st, A,
                           Bhi, Blo, C, M, K, N);
    return hipGetLastError();
}

}  // namespace snrt
