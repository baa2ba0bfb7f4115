// Scattering products C = A X in FP32 / FP64 on the vector ALUs: the dense kernel S = Psi B
// of eq. SNEqns (S_cq = sum_p psi_cp B[p][q], B[p][q] = w_p K[q][p]) and the two skinny
// products of the moment-projected form of eq. SNEqns2.  A [M][K], X [K][N], C [M][N].
//
// A plain LDS-tiled product: 64 x 64 output tile per 256-thread block, 4 x 4 outputs per
// thread, K staged in chunks of 16.  M (cells) runs over blockIdx.x, N (ordinates) over
// blockIdx.y.  Every load is bounds-checked, so any nq and any number of cells work.
// This is the FP32 precision mode and the FP64 parity template; the BF16 hi+lo MFMA
// product is the fast path.
#include "snrt_internal.h"

namespace snrt {

namespace {

constexpr int BM = 64, BN = 64, BK = 16;

template <typename T>
__global__ __launch_bounds__(256) void k_gemm_simple(const T* __restrict__ A,
                                                    const T* __restrict__ B, T* __restrict__ C,
                                                    int64_t M, int32_t N, int32_t K)
{
    __shared__ T As[BK][BM + 1];
    __shared__ T Bs[BK][BN + 1];
    const int tid = threadIdx.x;
    const int tx = tid % 16, ty = tid / 16;
    const int64_t m0 = (int64_t)blockIdx.x * BM;
    const int n0 = blockIdx.y * BN;
    T acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = T(0);

    for (int k0 = 0; k0 < K; k0 += BK) {
        // A tile: BM x BK, 4 elements per thread
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = tid + e * 256;
            const int r = idx / BK, kk = idx % BK;
            const int64_t gm = m0 + r;
            const int gk = k0 + kk;
            As[kk][r] = (gm < M && gk < K) ? A[gm * K + gk] : T(0);
        }
        // B tile: BK x BN
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = tid + e * 256;
            const int kk = idx / BN, cn = idx % BN;
            const int gk = k0 + kk, gn = n0 + cn;
            Bs[kk][cn] = (gk < K && gn < N) ? B[(int64_t)gk * N + gn] : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; ++kk) {
            T a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t gm = m0 + ty * 4 + i;
        if (gm >= M) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int gn = n0 + tx * 4 + j;
            if (gn < N) C[gm * N + gn] = acc[i][j];
        }
    }
}

template <typename T>
hipError_t launch(const T* A, const T* B, T* C, int64_t M, int32_t K, int32_t N, hipStream_t st) {
    if (M == 0 || N == 0) return hipSuccess;
    dim3 grid((unsigned)((M + BM - 1) / BM), (unsigned)((N + BN - 1) / BN));
    hipLaunchKernelGGL(k_gemm_simple<T>, grid, dim3(256), 0, st, A, B, C, M, N, K);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm32(const float* A, const float* B, float* C, int64_t M, int32_t K,
                         int32_t N, hipStream_t st) {
    return launch<float>(A, B, C, M, K, N, st);
}

hipError_t launch_gemm64(const double* A, const double* B, double* C, int64_t M, int32_t K,
                         int32_t N, hipStream_t st) {
    return launch<double>(A, B, C, M, K, N, st);
}

}  // namespace snrt
