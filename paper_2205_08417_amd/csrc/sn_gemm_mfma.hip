// Scattering products C = A X on the CDNA4 matrix cores (kernels and launchers; the
// block-tile core, its split-precision scheme and its tiling are in sn_gemm_core.h).
#include "sn_gemm_core.h"

namespace snrt {

namespace {

using namespace gemm;

// Blocks [0, nmain) are 256 x 256 tiles of the first M1 rows; blocks [nmain, grid) are
// TM x TN tiles of the remaining rows (none when nmain == grid).  Blocks are dispatched in
// order, so the small tiles fill the compute units as the full ones finish.
template <bool F16, int P, int MBN, int TM, int TN, int TFD, bool STAGGER>
__device__ __forceinline__ void gemm_grid(const float* __restrict__ A,
                                          const uint16_t* __restrict__ Bhi,
                                          const uint16_t* __restrict__ Blo, float* __restrict__ C,
                                          int64_t M1, int64_t M, int32_t K, int32_t N,
                                          int32_t ldc, const int32_t* __restrict__ rexp,
                                          int32_t eb, int64_t nmain, const GemmEpi& epi)
{
    constexpr int NP = P == 3 ? 4 : P == 2 ? 3 : 2;
    __shared__ __attribute__((aligned(16))) uint16_t lds[2 * NP * kPlane];
    const int64_t b = blockIdx.x;
    if (b < nmain) {
        // 256 x 256 tiles keep one chunk in flight (their multiply covers the load latency
        // and their accumulators leave no room for more); 256 x 128 tiles keep two
        // columns past ldc (the zero padding of X) are not stored
        gemm_block<P, 256, MBN, MBN == 256 ? 1 : 2, STAGGER, F16>(
            A, Bhi, Blo, M1, K, N, rexp, eb, xcd_remap(b, nmain), lds,
            [&](auto& acc, const TileInfo& t, auto row_of, auto exp_of) {
                epilogue_any(epi, acc, C, M1, ldc, t.n0 + t.wn, t.lane, row_of, exp_of);
            });
    } else {
        // nmain is a multiple of the XCD count, so the remap of the tail stays XCD-aware
        const int64_t nt = (int64_t)gridDim.x - nmain;
        const GemmEpi et = epi_rows_from(epi, M1);
        gemm_block<P, TM, TN, TFD, STAGGER, F16>(
            A + M1 * K, Bhi, Blo, M - M1, K, N, F16 ? rexp + M1 : rexp, eb,
            xcd_remap(b - nmain, nt), lds,
            [&](auto& acc, const TileInfo& t, auto row_of, auto exp_of) {
                epilogue_any(et, acc, C + M1 * ldc, M - M1, ldc, t.n0 + t.wn, t.lane, row_of,
                             exp_of);
            });
    }
}

template <int P, int MBN, int TM, int TN, int TFD, bool STAGGER>
__global__ __launch_bounds__(kThreads) void k_gemm_bf16(const float* __restrict__ A,
                                                        const uint16_t* __restrict__ Bhi,
                                                        const uint16_t* __restrict__ Blo,
                                                        float* __restrict__ C, int64_t M1,
                                                        int64_t M, int32_t K, int32_t N,
                                                        int32_t ldc, int64_t nmain,
                                                        GemmEpi epi)
{
    gemm_grid<false, P, MBN, TM, TN, TFD, STAGGER>(A, Bhi, Blo, C, M1, M, K, N, ldc, nullptr, 0,
                                                   nmain, epi);
}

// The FP16 hi+lo product (three products) with per-row exponents rexp of A and exponent eb
// of X.
template <int MBN, int TM, int TN, int TFD, bool STAGGER>
__global__ __launch_bounds__(kThreads) void k_gemm_f16(const float* __restrict__ A,
                                                       const uint16_t* __restrict__ Bhi,
                                                       const uint16_t* __restrict__ Blo,
                                                       float* __restrict__ C, int64_t M1,
                                                       int64_t M, int32_t K, int32_t N,
                                                       int32_t ldc,
                                                       const int32_t* __restrict__ rexp,
                                                       int32_t eb, int64_t nmain, GemmEpi epi)
{
    gemm_grid<true, 3, MBN, TM, TN, TFD, STAGGER>(A, Bhi, Blo, C, M1, M, K, N, ldc, rexp, eb,
                                                  nmain, epi);
}

// Row exponents of A [M][K] for the FP16 product: e_r with max_k |A[r][k]| * 2^e_r in
// [2^13, 2^14) (frexp of the row maximum m = f 2^E, f in [0.5, 1): e_r = 14 - E); 0 for a row
// of zeros or with a non-finite entry.  One wavefront per row, K % 4 == 0.
__global__ __launch_bounds__(256) void k_row_exp_f16(const float* __restrict__ A, int64_t M,
                                                     int32_t K, int32_t* __restrict__ rexp)
{
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); r < M; r += nw) {
        const f32x4* row = reinterpret_cast<const f32x4*>(A + r * K);
        float mx = 0.0f;
        for (int k = lane; k < K / 4; k += 64) {
            const f32x4 v = row[k];
            mx = fmaxf(mx, fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3]))));
            // a NaN anywhere makes the row's exponent 0 (fmaxf would drop it)
            if (v[0] != v[0] || v[1] != v[1] || v[2] != v[2] || v[3] != v[3]) mx = INFINITY;
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
        if (lane == 0) {
            int E = 0;
            (void)__builtin_frexpf(mx, &E);
            rexp[r] = (mx > 0.0f && mx < INFINITY) ? 14 - E : 0;
        }
    }
}

// ---------------------------------------------------------------------------------------
// FP32 product on the matrix cores (v_mfma_f32_32x32x2_f32): the FP32 precision mode.  Same
// block structure as the BF16 kernel (8 waves as 2 x 4, 32 x 32 MFMA tiles, K in chunks of
// 32 through two LDS stages), with FP32 planes [rows][32] and no operand split.  One MFMA
// takes two k values per row (lanes 0-31 and 32-63); lane half h carries k = 16h + s at
// step s, so each lane's 16 k values of a chunk are contiguous and one 16-byte LDS read feeds
// four steps (the accumulation order differs from a sequential k sum only by rounding).
// Planes store the 16-byte granule g of row r at position g ^ ((r >> 1) & 7): 16
// consecutive rows then cover the 256 bytes of LDS banks once.
__device__ __forceinline__ int swz8(int r, int g) { return g ^ ((r >> 1) & 7); }

typedef float f32x16v __attribute__((ext_vector_type(16)));

template <int BM, int BN, int FD>
__device__ __forceinline__ void gemm_block_f32(const float* __restrict__ A,
                                               const float* __restrict__ Bt,
                                               float* __restrict__ C, int64_t M, int32_t K,
                                               int32_t N, int64_t lb, float* lds,
                                               const GemmEpi& epi)
{
    static_assert(BM == 64 || BM == 128 || BM == 256, "block rows");
    static_assert(BN == 128 || BN == 256, "block columns");
    constexpr int IM = BM / 64, JN = BN / 128;
    constexpr int AV = BM / 64;                 // A float4 per thread per chunk
    constexpr int BVf = BN / 64;                // B float4 per thread per chunk
    constexpr int kPlaneF = 256 * BK;           // floats of one plane (32 KB)

    const int nN = N / BN;
    const int64_t m0 = (lb / nN) * BM;
    const int n0 = (int)(lb % nN) * BN;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wm = (wave >> 2) * (BM / 2);
    const int wn = (wave & 3) * (BN / 4);
    const int nk = K / BK;

    const uint32_t a_bytes = (uint32_t)((M - m0 < BM ? M - m0 : BM) * (int64_t)K * 4);
    const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(A + m0 * K), 0, (int32_t)a_bytes, kRsrcWord3);

    f32x4 ga[FD][AV], gb[FD][BVf];
    auto fetch = [&](int kc, int slot) {
#pragma unroll
        for (int e = 0; e < AV; ++e) {
            const int p = tid + e * kThreads;
            const int r = p >> 3, g = p & 7;
            i32x4 v = __builtin_amdgcn_raw_buffer_load_b128(
                ra, (uint32_t)((r * K + kc * BK + g * 4) * 4), 0, 0);
            ga[slot][e] = __builtin_bit_cast(f32x4, v);
        }
        const size_t tile = ((size_t)kc * N + n0) * BK;
#pragma unroll
        for (int e = 0; e < BVf; ++e) {
            const int p = tid + e * kThreads;
            gb[slot][e] = *reinterpret_cast<const f32x4*>(Bt + tile + (size_t)p * 4);
        }
    };
    auto stash = [&](int s, int slot) {
        float* Ap = lds + (s * 2 + 0) * kPlaneF;
        float* Bp = lds + (s * 2 + 1) * kPlaneF;
#pragma unroll
        for (int e = 0; e < AV; ++e) {
            const int p = tid + e * kThreads;
            const int r = p >> 3, g = p & 7;
            *reinterpret_cast<f32x4*>(&Ap[r * BK + swz8(r, g) * 4]) = ga[slot][e];
        }
#pragma unroll
        for (int e = 0; e < BVf; ++e) {
            const int p = tid + e * kThreads;    // X is stored in the plane's order
            *reinterpret_cast<f32x4*>(&Bp[p * 4]) = gb[slot][e];
        }
    };

    f32x16v acc[IM][JN];
#pragma unroll
    for (int i = 0; i < IM; ++i)
#pragma unroll
        for (int j = 0; j < JN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    const int fr = lane & 31, half = lane >> 5;
    fetch(0, 0);
    stash(0, 0);
#pragma unroll
    for (int d = 1; d <= FD; ++d)
        if (d < nk) fetch(d, d % FD);
    for (int kb = 0; kb < nk; kb += FD) {
#pragma unroll
        for (int u = 0; u < FD; ++u) {
            const int kc = kb + u;
            if (kc >= nk) break;
            const int s = kc & 1;
            __syncthreads();             // chunk kc staged; the idle stage is free again
            if (kc + 1 < nk) stash(s ^ 1, (u + 1) % FD);
            if (kc + 1 + FD < nk) fetch(kc + 1 + FD, (u + 1) % FD);
            const float* Ap = lds + (s * 2 + 0) * kPlaneF;
            const float* Bp = lds + (s * 2 + 1) * kPlaneF;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int g = 4 * half + t;      // this lane's k = 16 half + 4 t + [0, 4)
                f32x4 a[IM], b[JN];
#pragma unroll
                for (int i = 0; i < IM; ++i) {
                    const int r = wm + i * 32 + fr;
                    a[i] = *reinterpret_cast<const f32x4*>(&Ap[r * BK + swz8(r, g) * 4]);
                }
#pragma unroll
                for (int j = 0; j < JN; ++j) {
                    const int n = wn + j * 32 + fr;
                    b[j] = *reinterpret_cast<const f32x4*>(&Bp[n * BK + swz8(n, g) * 4]);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int i = 0; i < IM; ++i)
#pragma unroll
                        for (int j = 0; j < JN; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i][q], b[j][q],
                                                                             acc[i][j], 0, 0, 0);
            }
        }
    }

    auto row_of = [&](int i, int r) -> int64_t {
        return m0 + wm + i * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
    };
    auto exp_of = [](int64_t) -> int { return 0; };
    (void)fr;
    epilogue_any(epi, acc, C, M, N, n0 + wn, lane, row_of, exp_of);
}

template <int MBN, int TM, int TN, int TFD>
__global__ __launch_bounds__(kThreads) void k_gemm_f32(const float* __restrict__ A,
                                                       const float* __restrict__ Bt,
                                                       float* __restrict__ C, int64_t M1,
                                                       int64_t M, int32_t K, int32_t N,
                                                       int64_t nmain, GemmEpi epi)
{
    __shared__ __attribute__((aligned(16))) float lds[2 * 2 * 256 * BK];
    const int64_t b = blockIdx.x;
    if (b < nmain) {
        gemm_block_f32<256, MBN, MBN == 256 ? 1 : 2>(A, Bt, C, M1, K, N, xcd_remap(b, nmain),
                                                     lds, epi);
    } else {
        const int64_t nt = (int64_t)gridDim.x - nmain;
        gemm_block_f32<TM, TN, TFD>(A + M1 * K, Bt, C + M1 * N, M - M1, K, N,
                                    xcd_remap(b - nmain, nt), lds, epi_rows_from(epi, M1));
    }
}

// X [K][N] FP32 in the FP32 plane order: the 128-byte row (kc, n) holds X[kc*32 + k][n],
// k = 0..31, as eight 16-byte granules with granule g at position g ^ ((n >> 1) & 7).
__global__ __launch_bounds__(256) void k_tile_f32(const float* __restrict__ B,
                                                  float* __restrict__ out, int32_t K, int32_t N)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)K * N) return;
    const int pos = (int)(i % BK);
    const int64_t t = i / BK;
    const int n = (int)(t % N);
    const int kc = (int)(t / N);
    const int k = swz8(n, pos >> 2) * 4 + (pos & 3);
    out[i] = B[(int64_t)(kc * BK + k) * N + n];
}

// Tiled halves of X [K][N] in the LDS plane order: the 64-byte row (kc, n) holds
// X[kc*32 + kk][n], kk = 0..31, as four 16-byte granules with granule g at position
// g ^ ((n >> 2) & 3); hi = bf16(X), lo = bf16(X - hi).
__global__ __launch_bounds__(256) void k_split(const float* __restrict__ B, uint16_t* __restrict__ hi,
                                               uint16_t* __restrict__ lo, int32_t K, int32_t N)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)K * N) return;
    const int pos = (int)(i % BK);
    const int64_t t = i / BK;
    const int n = (int)(t % N);
    const int kc = (int)(t / N);
    const int kk = swz(n, pos >> 3) * 8 + (pos & 7);
    const float x = B[(int64_t)(kc * BK + kk) * N + n];
    const uint32_t h = bf16_rne_bits(x);
    hi[i] = (uint16_t)h;
    lo[i] = (uint16_t)bf16_rne_bits(x - bf16_to_f32(h));
}

// FP16 halves of X [K][N] scaled by 2^eb, in the same tiled plane order as k_split.
__global__ __launch_bounds__(256) void k_split_f16(const float* __restrict__ B,
                                                   uint16_t* __restrict__ hi,
                                                   uint16_t* __restrict__ lo, int32_t K, int32_t N,
                                                   int32_t eb)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)K * N) return;
    const int pos = (int)(i % BK);
    const int64_t t = i / BK;
    const int n = (int)(t % N);
    const int kc = (int)(t / N);
    const int kk = swz(n, pos >> 3) * 8 + (pos & 7);
    const float x = __builtin_ldexpf(B[(int64_t)(kc * BK + kk) * N + n], eb);
    const _Float16 h = (_Float16)x;
    hi[i] = f16_bits(h);
    lo[i] = f16_bits((_Float16)(x - (float)h));
}

}  // namespace

hipError_t launch_split_f16(const float* B, uint16_t* hi, uint16_t* lo, int32_t K, int32_t N,
                            int32_t eb, hipStream_t st) {
    if (K % BK != 0 || N % 128 != 0) return hipErrorNotSupported;
    const int64_t n = (int64_t)K * N;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_split_f16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, B, hi,
                       lo, K, N, eb);
    return hipGetLastError();
}

hipError_t launch_tile_f32(const float* B, float* out, int32_t K, int32_t N, hipStream_t st) {
    if (K % BK != 0 || N % 128 != 0) return hipErrorNotSupported;
    const int64_t n = (int64_t)K * N;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, B, out,
                       K, N);
    return hipGetLastError();
}

hipError_t launch_split_bf16(const float* B, uint16_t* hi, uint16_t* lo, int32_t K, int32_t N,
                             hipStream_t st) {
    if (K % BK != 0 || N % 128 != 0) return hipErrorNotSupported;
    const int64_t n = (int64_t)K * N;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_split, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, B, hi, lo, K, N);
    return hipGetLastError();
}

// Compute units of the current device (cached per device).
int device_cu_count() {
    static int cache[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cache[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            n <= 0)
            n = 256;
        cache[dev] = n;
    }
    return cache[dev];
}

// products 1..3: BF16; 0: the FP16 three-product form (rexp, eb).
template <int MBN, int TM, int TN>
hipError_t launch_split(const float* A, const uint16_t* Bhi, const uint16_t* Blo, float* C,
                        int64_t M1, int64_t M, int32_t K, int32_t N, int32_t ldc, int products,
                        const int32_t* rexp, int32_t eb, hipStream_t st, const GemmEpi& epi) {
    const int64_t nmain = ((M1 + 255) / 256) * (N / MBN);
    const int64_t ntail = ((M - M1 + TM - 1) / TM) * (N / TN);
    const dim3 grid((unsigned)(nmain + ntail));
    auto go = [&](auto p_c, auto stagger_c) {
        constexpr int PP = decltype(p_c)::value;
        constexpr bool SG = decltype(stagger_c)::value;
        if constexpr (PP == 0)
            hipLaunchKernelGGL((k_gemm_f16<MBN, TM, TN, 4, SG>), grid, dim3(kThreads), 0, st, A,
                               Bhi, Blo, C, M1, M, K, N, ldc, rexp, eb, nmain, epi);
        else
            hipLaunchKernelGGL((k_gemm_bf16<PP, MBN, TM, TN, 4, SG>), grid, dim3(kThreads), 0,
                               st, A, Bhi, Blo, C, M1, M, K, N, ldc, nmain, epi);
        return hipGetLastError();
    };
    // the staggered phases pay on the square products of the dense kernel (4-5 % measured);
    // on the skinny moment products (an inner or outer width of 128) they cost 3 %
    const bool stagger = tune().gemm_stagger && K >= 256 && N >= 256;
    auto by_stagger = [&](auto p_c) {
        return stagger ? go(p_c, std::true_type{}) : go(p_c, std::false_type{});
    };
    if (products == 0) return by_stagger(std::integral_constant<int, 0>{});
    if (products == 3) return by_stagger(std::integral_constant<int, 3>{});
    if (products == 2) return by_stagger(std::integral_constant<int, 2>{});
    return by_stagger(std::integral_constant<int, 1>{});
}

// One 256 x 256 block (256 x 128 when N is an odd multiple of 128) per compute unit and
// round (128 KB of LDS each).  When the last round would be mostly empty, its rows run as
// smaller blocks: 64 x 128 (an eighth of a 256 x 256 block) if they then fill one round,
// else 64 x 256 (a quarter) if those fill one round; a small block takes about half the time
// of a full one (measured), so a fuller last round stays as it is.  With 256 x 128 blocks
// only the quarter (64 x 128) applies.
GemmPlan gemm_plan(int64_t M, int32_t N) {
    const bool wide = N % 256 == 0;
    const int64_t nN = wide ? N / 256 : N / 128;
    const int64_t tiles = ((M + 255) / 256) * nN;
    const int64_t cu = device_cu_count();
    const int64_t rem = tiles % cu;
    const bool level = tiles > cu && rem != 0 && cu % kNumXcd == 0;
    const bool eighth = wide && level && rem * 8 <= cu;
    const bool quarter = !eighth && level && rem * 4 <= cu;
    const int64_t rows1 = std::min<int64_t>(((tiles - rem) / nN) * 256, M);
    GemmPlan p;
    p.mbn = wide ? 256 : 128;
    p.tm = 64;
    p.tn = (wide && !eighth) ? 256 : 128;
    p.rows1 = (eighth || quarter) ? rows1 : M;
    return p;
}

hipError_t launch_row_exp_f16(const float* A, int64_t M, int32_t K, int32_t* rexp,
                              hipStream_t st) {
    if (M == 0) return hipSuccess;
    if (!rexp || K % 4 != 0) return hipErrorNotSupported;
    const int64_t want = (M + 3) / 4;
    const unsigned nb = (unsigned)std::min<int64_t>(want, (int64_t)device_cu_count() * 8);
    hipLaunchKernelGGL(k_row_exp_f16, dim3(nb), dim3(256), 0, st, A, M, K, rexp);
    return hipGetLastError();
}

// The shape policy of both low-precision products (products 1..3: BF16; 0: FP16 x3).
hipError_t launch_gemm_lp(const float* A, const uint16_t* Bhi, const uint16_t* Blo, float* C,
                          int64_t M, int32_t K, int32_t N, int32_t ldc, int products,
                          const int32_t* rexp, int32_t eb, hipStream_t st, const GemmEpi& epi) {
    if (M == 0) return hipSuccess;
    if (products < 0 || products > 3) return hipErrorInvalidValue;
    if (K % BK != 0 || N % 128 != 0 || K == 0 || ldc <= 0 || ldc > N)
        return hipErrorNotSupported;
    const GemmPlan p = gemm_plan(M, N);
    if (p.mbn == 128)
        return launch_split<128, 64, 128>(A, Bhi, Blo, C, p.rows1, M, K, N, ldc, products,
                                          rexp, eb, st, epi);
    if (p.tn == 128)
        return launch_split<256, 64, 128>(A, Bhi, Blo, C, p.rows1, M, K, N, ldc, products,
                                          rexp, eb, st, epi);
    return launch_split<256, 64, 256>(A, Bhi, Blo, C, p.rows1, M, K, N, ldc, products, rexp,
                                      eb, st, epi);
}

hipError_t launch_gemm_bf16(const float* A, const uint16_t* Bhi, const uint16_t* Blo, float* C,
                            int64_t M, int32_t K, int32_t N, int32_t ldc, int products,
                            hipStream_t st, const GemmEpi& epi) {
    if (products < 1 || products > 3) return hipErrorInvalidValue;
    return launch_gemm_lp(A, Bhi, Blo, C, M, K, N, ldc, products, nullptr, 0, st, epi);
}

hipError_t launch_gemm_f16x3(const float* A, const uint16_t* Bhi, const uint16_t* Blo, float* C,
                             int64_t M, int32_t K, int32_t N, int32_t ldc, int32_t* rexp,
                             int32_t eb, hipStream_t st, const GemmEpi& epi) {
    if (M == 0) return hipSuccess;
    if (!rexp || K % BK != 0 || K == 0) return hipErrorNotSupported;
    const hipError_t e = launch_row_exp_f16(A, M, K, rexp, st);
    if (e != hipSuccess) return e;
    return launch_gemm_lp(A, Bhi, Blo, C, M, K, N, ldc, 0, rexp, eb, st, epi);
}

template <int MBN, int TM, int TN>
hipError_t launch_f32_split(const float* A, const float* Bt, float* C, int64_t M1, int64_t M,
                            int32_t K, int32_t N, hipStream_t st, const GemmEpi& epi) {
    const int64_t nmain = ((M1 + 255) / 256) * (N / MBN);
    const int64_t ntail = ((M - M1 + TM - 1) / TM) * (N / TN);
    hipLaunchKernelGGL((k_gemm_f32<MBN, TM, TN, 4>), dim3((unsigned)(nmain + ntail)),
                       dim3(kThreads), 0, st, A, Bt, C, M1, M, K, N, nmain, epi);
    return hipGetLastError();
}

hipError_t launch_gemm_f32mfma(const float* A, const float* Bt, float* C, int64_t M, int32_t K,
                               int32_t N, hipStream_t st, const GemmEpi& epi) {
    if (M == 0) return hipSuccess;
    if (K % BK != 0 || N % 128 != 0 || K == 0) return hipErrorNotSupported;
    // the same block shapes and last-round policy as the BF16 product
    const bool wide = N % 256 == 0;
    const int64_t nN = wide ? N / 256 : N / 128;
    const int64_t tiles = ((M + 255) / 256) * nN;
    const int64_t cu = device_cu_count();
    const int64_t rem = tiles % cu;
    const bool level = tiles > cu && rem != 0 && cu % kNumXcd == 0;
    const bool eighth = wide && level && rem * 8 <= cu;
    const bool quarter = !eighth && level && rem * 4 <= cu;
    const int64_t rows1 = std::min<int64_t>(((tiles - rem) / nN) * 256, M);
    if (!wide)
        return quarter ? launch_f32_split<128, 64, 128>(A, Bt, C, rows1, M, K, N, st, epi)
                       : launch_f32_split<128, 64, 128>(A, Bt, C, M, M, K, N, st, epi);
    if (eighth) return launch_f32_split<256, 64, 128>(A, Bt, C, rows1, M, K, N, st, epi);
    if (quarter) return launch_f32_split<256, 64, 256>(A, Bt, C, rows1, M, K, N, st, epi);
    return launch_f32_split<256, 64, 256>(A, Bt, C, M, M, K, N, st, epi);
}

}  // namespace snrt
