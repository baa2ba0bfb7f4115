// Dense scattering product S = Psi B on the CDNA4 matrix cores (eq. SNEqns with a dense
// kernel: S_cq = sum_p psi_cp B[p][q], B[p][q] = w_p K[q][p]).
//
// Split precision: every FP32 operand x is written as hi + lo with hi = bf16(x) and
// lo = bf16(x - hi) (round to nearest even; x - hi is exact in FP32), and the product is
// accumulated in FP32 as  A_hi B_hi + A_hi B_lo + A_lo B_hi  (the lo*lo term, below 2^-16
// relative, is dropped).  The single-product mode keeps only A_hi B_hi.
//
// Tiling for v_mfma_f32_32x32x16_bf16 (64-lane wavefronts):
//   block tile 128 (cells) x 256 (ordinates), 8 waves as 2 x 4, each wave 64 x 64 =
//   2 x 2 MFMA tiles with FP32 accumulators; K staged through LDS in chunks of 32.
//   A (Psi, FP32 rows) is split while it is copied to LDS; B arrives pre-split and
//   transposed ([n][k] BF16) so that both operands are read from LDS as 16-byte
//   fragments along K.  LDS rows are padded to 40 elements (80 B), which keeps the eight
//   16-byte reads of each quarter-wave on distinct banks.
//   The next chunk's global data is fetched into registers while the current chunk is
//   multiplied.  Consecutive logical blocks share an A row block (its N tiles), and the
//   XCD-aware block order keeps them on one XCD so A is fetched from HBM once.
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

constexpr int BM = 128, BN = 256, BK = 32, LDSK = BK + 8;
constexpr int kThreads = 512;
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

template <bool THREE>
__global__ __launch_bounds__(kThreads) void k_gemm_bf16(const float* __restrict__ A,
                                                        const uint16_t* __restrict__ Bhi,
                                                        const uint16_t* __restrict__ Blo,
                                                        float* __restrict__ C, int64_t M,
                                                        int32_t nq)
{
    __shared__ __attribute__((aligned(16))) uint16_t sAh[BM * LDSK];
    __shared__ __attribute__((aligned(16))) uint16_t sAl[BM * LDSK];
    __shared__ __attribute__((aligned(16))) uint16_t sBh[BN * LDSK];
    __shared__ __attribute__((aligned(16))) uint16_t sBl[THREE ? BN * LDSK : 8];

    const int nN = nq / BN;
    const int64_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t m0 = (lb / nN) * BM;
    const int n0 = (int)(lb % nN) * BN;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wm = (wave >> 2) * 64;        // wave tile origin inside the block tile
    const int wn = (wave & 3) * 64;

    // A rows as a buffer resource: rows past M read as zero
    const uint32_t a_bytes = (uint32_t)((M - m0 < BM ? M - m0 : BM) * (int64_t)nq * 4);
    const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(A + m0 * nq), 0, (int32_t)a_bytes, kRsrcWord3);

    // global -> register staging: A 128 x 32 floats = 1024 float4 (2 per thread);
    // B 256 x 32 bf16 per half = 1024 16-byte pieces per half (2 per thread per half)
    f32x4 ga[2];
    u32x4 gbh[2], gbl[2];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int idx = tid + e * kThreads;
            const int r = idx >> 3, k4 = idx & 7;
            i32x4 v = __builtin_amdgcn_raw_buffer_load_b128(
                ra, (uint32_t)((r * nq + k0 + k4 * 4) * 4), 0, 0);
            ga[e] = __builtin_bit_cast(f32x4, v);
        }
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int idx = tid + e * kThreads;
            const int n = idx >> 2, k8 = idx & 3;
            const size_t off = (size_t)(n0 + n) * nq + k0 + k8 * 8;
            gbh[e] = *reinterpret_cast<const u32x4*>(Bhi + off);
            if constexpr (THREE) gbl[e] = *reinterpret_cast<const u32x4*>(Blo + off);
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int idx = tid + e * kThreads;
            const int r = idx >> 3, k4 = idx & 7;
            uint32_t hi[2], lo[2];
            split4(ga[e], hi, lo);
            *reinterpret_cast<uint2*>(&sAh[r * LDSK + k4 * 4]) = make_uint2(hi[0], hi[1]);
            *reinterpret_cast<uint2*>(&sAl[r * LDSK + k4 * 4]) = make_uint2(lo[0], lo[1]);
        }
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int idx = tid + e * kThreads;
            const int n = idx >> 2, k8 = idx & 3;
            *reinterpret_cast<u32x4*>(&sBh[n * LDSK + k8 * 8]) = gbh[e];
            if constexpr (THREE) *reinterpret_cast<u32x4*>(&sBl[n * LDSK + k8 * 8]) = gbl[e];
        }
    };

    f32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    const int fr = lane & 31;            // fragment row / column
    const int fk = (lane >> 5) * 8;      // fragment K offset
    fetch(0);
    for (int k0 = 0; k0 < nq; k0 += BK) {
        __syncthreads();                 // previous chunk's fragments are consumed
        stash();
        __syncthreads();
        if (k0 + BK < nq) fetch(k0 + BK);
#pragma unroll
        for (int ks = 0; ks < BK; ks += 16) {
            bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int ar = (wm + t * 32 + fr) * LDSK + ks + fk;
                const int bc = (wn + t * 32 + fr) * LDSK + ks + fk;
                ah[t] = *reinterpret_cast<const bf16x8*>(&sAh[ar]);
                bh[t] = *reinterpret_cast<const bf16x8*>(&sBh[bc]);
                if constexpr (THREE) {
                    al[t] = *reinterpret_cast<const bf16x8*>(&sAl[ar]);
                    bl[t] = *reinterpret_cast<const bf16x8*>(&sBl[bc]);
                }
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
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

    // epilogue: accumulator i of lane l is row (i/4)*8 + (l/32)*4 + i%4, column l%32
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int col = n0 + wn + j * 32 + fr;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t row = m0 + wm + i * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
                if (row < M) C[row * nq + col] = acc[i][j][r];
            }
        }
}

// hi[n][k] = bf16(B[k][n]), lo[n][k] = bf16(B[k][n] - hi): transposed BF16 halves
__global__ __launch_bounds__(256) void k_split(const float* __restrict__ B, uint16_t* __restrict__ hi,
                                               uint16_t* __restrict__ lo, int32_t nq)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)nq * nq) return;
    const int n = (int)(i / nq), k = (int)(i % nq);
    const float x = B[(int64_t)k * nq + n];
    const uint32_t h = bf16_rne_bits(x);
    hi[i] = (uint16_t)h;
    lo[i] = (uint16_t)bf16_rne_bits(x - bf16_to_f32(h));
}

}  // namespace

hipError_t launch_split_bf16(const float* B, uint16_t* hi, uint16_t* lo, int32_t nq,
                             hipStream_t st) {
    const int64_t n = (int64_t)nq * nq;
    hipLaunchKernelGGL(k_split, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, B, hi, lo, nq);
    return hipGetLastError();
}

hipError_t launch_gemm_bf16(const float* A, const uint16_t* Bhi, const uint16_t* Blo, float* C,
                            int64_t M, int32_t nq, bool three_products, hipStream_t st) {
    if (M == 0) return hipSuccess;
    if (nq % BN != 0) return hipErrorNotSupported;
    const int64_t blocks = ((M + BM - 1) / BM) * (nq / BN);
    if (three_products)
        hipLaunchKernelGGL(k_gemm_bf16<true>, dim3((unsigned)blocks), dim3(kThreads), 0, st, A,
                           Bhi, Blo, C, M, nq);
    else
        hipLaunchKernelGGL(k_gemm_bf16<false>, dim3((unsigned)blocks), dim3(kThreads), 0, st, A,
                           Bhi, Blo, C, M, nq);
    return hipGetLastError();
}

}  // namespace snrt
