// The mode-space IMEX combine in one launch with its product (kernel templates in
// sn_step_fused.h).
#include "sn_step_fused.h"

namespace snrt {
namespace fused {
namespace {

hipError_t launch_gemm_combine_impl(const float* A, const uint16_t* Bhi, const uint16_t* Blo,
                                    int64_t M, int32_t K, int32_t N, int products,
                                    const int32_t* rexp, int32_t eb, const CombineEpi& ce,
                                    hipStream_t st)
{
    if (M == 0) return hipSuccess;
    if (products < 0 || products > 3) return hipErrorInvalidValue;
    if (K % 32 != 0 || K == 0 || N % 256 != 0 || N != ce.nq || M != ce.nc ||
        (products == 0 && !rexp))
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
        hipLaunchKernelGGL((k_gemm_combine<PP == 0, PP == 0 ? 3 : PP, 64, TN, SG>), grid,
                           dim3(gemm::kThreads), 0, st, A, Bhi, Blo, p.rows1, M, K, N, rexp, eb,
                           nmain, ce);
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

}  // namespace
}  // namespace fused

hipError_t launch_gemm_combine(const float* A, const uint16_t* Bhi, const uint16_t* Blo,
                               int64_t M, int32_t K, int32_t N, int products,
                               const int32_t* rexp, int32_t eb, const CombineEpi& ce,
                               hipStream_t st) {
    return fused::launch_gemm_combine_impl(A, Bhi, Blo, M, K, N, products, rexp, eb, ce, st);
}

}  // namespace snrt
