// Internal types shared by the libsnrt translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/snrt.h"

namespace snrt {

constexpr int32_t kUnusedFace = INT32_MIN;
constexpr int kWave = 64;              // CDNA wavefront width
constexpr int kStepBlock = 256;        // 4 waves, one cell per wave
constexpr int kCellsPerBlock = kStepBlock / kWave;
constexpr int kNumXcd = 8;             // MI355X: 8 accelerator complex dies

// Per-cell geometry record, one 64-byte line: neighbours, n_ij (outward normal x length),
// 1/A_i and A_i.  An unused face slot points at the cell itself with a zero normal.
struct alignas(64) CellGeom32 {
    int32_t nbr[4];
    float n[4][2];
    float inv_area;
    float area;
    float pad[2];
};
static_assert(sizeof(CellGeom32) == 64, "one cache line per cell");

struct alignas(32) CellGeom64 {
    int32_t nbr[4];
    double n[4][2];
    double inv_area;
    double area;
    double pad[2];
};
static_assert(sizeof(CellGeom64) == 128, "two cache lines per cell");

// Reconstruction vectors of the second-order scheme, per face slot: r_own = face midpoint
// - own centroid, r_far = the same face's midpoint - the neighbour's centroid (zero for
// boundary faces, whose ghost value is not reconstructed, and for unused slots).
struct alignas(64) CellRecon32 {
    float r_own[4][2];
    float r_far[4][2];
};
static_assert(sizeof(CellRecon32) == 64, "one cache line per cell");

struct alignas(64) CellRecon64 {
    double r_own[4][2];
    double r_far[4][2];
};
static_assert(sizeof(CellRecon64) == 128, "two cache lines per cell");

// Right operand X [K][N] of a scattering product C = A X on the device, in every precision
// the products use: FP32 and FP64 row-major, and the BF16 or FP16 hi/lo parts for the MFMA
// kernel, with the columns zero-padded to Np (a multiple of 128) and tiled by K chunks of 32
// ([K/32][Np][32]); the FP16 parts hold X * 2^eb.
struct GemmOperand {
    int32_t K = 0, N = 0;
    int32_t Np = 0;           // padded width of the hi/lo parts
    int32_t eb = 0;           // FP16 scale exponent of X
    float* f32 = nullptr;
    double* f64 = nullptr;
    uint16_t* hi = nullptr;
    uint16_t* lo = nullptr;
    float* t32 = nullptr;     // FP32 in the MFMA kernel's tiled order (FP32 mode, if shaped)
};

// The scattering product as a chain of right operands, forward (S = Psi X0 [X1]) and adjoint
// (Lambda B^T):
//   dense kernel (chain 1):  X0 = B, B[p][q] = w_p K[q][p];  adjoint X0 = B^T;
//   moments (chain 2, eq. SNEqns2):  X0 = M^T [nq][mid] (w_q m_j(Omega_q)), X1 = (Sigma O)^T
//   [mid][nq] (sigma_l(j) m_j(Omega_q)); adjoint X0 = X1^T, X1 = X0^T.  mid = the moment
//   count (N+1)^2, padded with zero columns to a multiple of 32 (the K chunk) for the BF16
//   and FP16 MFMA kernels (unpadded in FP32).
struct DenseB {
    int32_t nq = 0;
    snrt_precision precision = SNRT_FP32;
    int32_t chain = 1;
    int32_t mid = 0;
    int32_t degree = -1;          // moment degree N (chain 2)
    // moment form: Sigma per moment index ([mid], zero past the (N+1)^2 moments) and
    // max |M O - I| over the moments (how exactly the quadrature integrates their products)
    float* msig32 = nullptr;
    double* msig64 = nullptr;
    double mo_err = 0.0;
    GemmOperand fwd[2], adj[2];
    // implicit form of a dense kernel (chain 1; snrt_scatter_prepare_implicit): K W =
    // V diag(lam) V^-1 as the operands imp[0] = V^-1 as [nq][nq] (x0[q][j] = V^-1[j][q]) and
    // imp[1] = (V diag(lam))^T (x1[j][q] = lam_j V[q][j]), with lam on the device
    bool implicit = false;
    GemmOperand imp[2];
    float* lam32 = nullptr;
    double* lam64 = nullptr;
    double imp_resid = 0.0;
};

// The eigendecomposition behind the implicit form (host, FP64): A [n][n] row-major with
// A[q][p] = K[q][p] w_p; fills lam [n] and the two product operands x0, x1 [n][n].  Returns
// SNRT_E_UNSUPPORTED (with the reason set) when A is not diagonally similar to a symmetric
// matrix or the decomposition fails its residual check.
snrt_status implicit_form(int n, const std::vector<double>& A, std::vector<double>& lam,
                          std::vector<double>& x0, std::vector<double>& x1, double* resid,
                          const char* fn);  // fn: the entry point named in error messages

}  // namespace snrt

struct snrt_mesh {
    int device = 0;
    int64_t nc = 0;
    int64_t nbf = 0;
    int32_t mf = 3;
    std::vector<int64_t> to_user;          // internal -> user
    snrt::CellGeom32* geom32 = nullptr;
    snrt::CellGeom64* geom64 = nullptr;
    int64_t* d_to_user = nullptr;          // device copy of to_user
    double* d_partial = nullptr;           // per-block partial sums for snrt_mass
    int64_t n_partial = 0;
    int num_cu = 256;                      // compute units of the device (launch shapes)
    // host copies kept for the second-order set-up (user order)
    std::vector<int32_t> face_nbr_user;    // [nc*mf]
    std::vector<double> centroid_user;     // [nc*2], empty if none was given
    snrt::CellRecon32* recon32 = nullptr;  // second-order reconstruction vectors (internal
    snrt::CellRecon64* recon64 = nullptr;  // order); NULL until face midpoints are set
};

struct snrt_quad {
    int device = 0;
    int32_t nq = 0;
    // FP32 ordinate table, 4 rows of nq: Omega_x, Omega_y, w, w/(4 pi)
    float* tab32 = nullptr;
    double* tab64 = nullptr;
    std::vector<double> w_host;
    std::vector<double> omega_host;        // [nq*3] unit directions (x, y, z)
};

// P_N system of degree N (Sec. 3.1 P_N closure, Sec. 4.3): the flux Jacobians, |A_x|,
// |A_y| (host copies, FP64) and the step's coefficient tables on the device, one per
// precision.  Degrees with an unrolled kernel (pn::has_fused_kernel<T>) use the packed
// table of that kernel (one value per structurally non-zero coefficient, halved, in
// pn::visit_ops order); the other degrees the dense table [nm][nmp][4] (X, Y, P, Q coefficient of input moment m for
// output k, halved, nmp = nm rounded up to a multiple of 16, the chunked kernel's step).
struct snrt_pn {
    int device = 0;
    int32_t degree = 0;
    int32_t nm = 0;
    int32_t nmp = 0;
    std::vector<double> ax, ay, ax_abs, ay_abs;   // [nm][nm]
    std::vector<double> sig;                      // sigma_l(j) per moment
    float* w32 = nullptr;
    double* w64 = nullptr;
    float* sig32 = nullptr;
    double* sig64 = nullptr;
    // the matrix-core step of degree pn::kFusedHighDegree: the A_x, A_y coefficients
    // (pn::SparseOps order), the class blocks' FP16 hi/lo operands [z parity][class][K step]
    // [hi, lo][lane][8] and their exponents [z parity][class]
    float* wsp32 = nullptr;
    uint16_t* wa16 = nullptr;
    int32_t* wae = nullptr;
};

struct snrt_scatter {
    int device = 0;
    bool dense = false;
    snrt::DenseB B;
};

namespace snrt {

// Launch-shape knobs of the persistent kernels and the BF16 product.  Defaults are the tuned
// values for MI355X.  SNRT_STEP_TUNE="<step>[,<second-order update>[,<adjoint>]]" overrides
// the blocks per CU of the three persistent sweeps, SNRT_GEMM_STAGGER=0 turns the staggered
// chunk order of the product off, SNRT_GEMM_EPILOGUE=0 the IMEX steps in the products'
// epilogues (separate passes instead), SNRT_PN_MFMA=0 the matrix-core class blocks of the
// degree-13 P_N step (all read once per process).
struct Tune {
    int step_blocks_per_cu = 3;
    int flux2_blocks_per_cu = 2;   // its larger per-cell footprint favours a narrower sweep
    int adjoint_blocks_per_cu = 7; // the adjoint's smaller workloads favour a wide grid
    bool gemm_stagger = true;      // staggered split/product phases in the BF16 product
    bool gemm_epilogue = true;     // IMEX per-cell steps in the products' epilogues
    bool pn_mfma = true;           // matrix-core class blocks in the degree-13 P_N step
    bool step_fused = true;        // dense step: the update in the product's epilogue
};
const Tune& tune();

void set_error(const std::string& msg);
snrt_status hip_fail(hipError_t e, const char* what);

// ---- host helpers shared by the ABI translation units
inline bool is_finite(double x) { return std::isfinite(x); }

template <typename T>
inline snrt_status dev_alloc(T** p, size_t count, const char* what) {
    *p = nullptr;
    if (count == 0) return SNRT_OK;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        set_error(std::string("device allocation failed for ") + what + ": " +
                  hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? SNRT_E_OOM : SNRT_E_HIP;
    }
    return SNRT_OK;
}

template <typename T>
inline snrt_status upload(T* dst, const T* src, size_t count, const char* what) {
    if (count == 0) return SNRT_OK;
    hipError_t e = hipMemcpy(dst, src, count * sizeof(T), hipMemcpyHostToDevice);
    return e == hipSuccess ? SNRT_OK : hip_fail(e, what);
}

inline void dev_free(void* p) {
    if (p) (void)hipFree(p);
}

inline snrt_status check_device(int dev, const char* what) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, what);
    if (cur != dev) {
        set_error(std::string(what) + ": handle belongs to device " + std::to_string(dev) +
                  " but device " + std::to_string(cur) + " is current");
        return SNRT_E_ARG;
    }
    return SNRT_OK;
}

inline bool ranges_overlap(const void* a, size_t abytes, const void* b, size_t bbytes) {
    const auto pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
    return pa < pb + bbytes && pb < pa + abytes;
}

inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Real spherical harmonics m_j (j = l^2 + l + k, degree <= N) at the unit direction (x, y, z).
void real_harmonics(int N, double x, double y, double z, double* out);

// Kernel launchers (return hipGetLastError() after the launch).
// The dose functional's term of a reverse rollout fused into the transposed step's output:
// lam_q += coeff (1/rho_c) g_dose[c] w_q (FP64; w: FP64 weights [nq]); g_dose NULL: none.
struct DoseAdj {
    const double* w = nullptr;
    double coeff = 0.0;
    const double* g_dose = nullptr;
};

struct StepArgs32 {
    const float *sigma_t, *sigma_s, *inv_rho, *source, *inflow;
    float inflow_scale, dt, alpha_t, alpha_s;
    int32_t neumann;
};
struct StepArgs64 {
    const double *sigma_t, *sigma_s, *inv_rho, *source, *inflow;
    double inflow_scale, dt, alpha_t, alpha_s;
    int32_t neumann;
};

// Argument checks of the FP32 step entry points (handles, devices, scalars, sizes, alignment,
// aliasing, the dense product's workspace) and the conversion of their arguments.
snrt_status check_step32(const char* fn, const snrt_mesh* m, const snrt_quad* q,
                         const snrt_scatter* sc, const snrt_step_args* a, const float* in,
                         float* out, void* ws, size_t ws_bytes);
StepArgs32 step_args32(const snrt_step_args* a);
// snrt_step_adjoint with the gradient contributions added to FP64 accumulators (the reverse
// pass of long rollouts, where FP32 accumulators would drift by rounding).
snrt_status step_adjoint32_acc64(const snrt_mesh* m, const snrt_quad* q, const snrt_scatter* sc,
                                 const snrt_step_args* a, const float* psi_n,
                                 const float* lam_np1, float* lam_n, double* g_t, double* g_s,
                                 double* g_r, void* ws, size_t ws_bytes, void* stream,
                                 const DoseAdj& da = DoseAdj());

// dose_part: with the fused dose, the [nc * items per row] FP64 weighted sums of psi_in
hipError_t launch_step32(const snrt_mesh& m, const snrt_quad& q, const StepArgs32& a,
                         const float* psi_in, float* psi_out, const float* S, hipStream_t st,
                         double* dose_part = nullptr);
// work items per state row of the FP32 step (row chunks of the dense step)
int32_t step_items_per_row(const snrt_quad& q, bool dense);
hipError_t launch_dose_fold(const snrt_mesh& m, const double* part, int32_t nch,
                            const float* inv_rho, double coeff, double* dose, hipStream_t st);
// nontemporal device copy of bytes / 16 16-byte vectors (bandwidth measurement)
hipError_t launch_stream_copy(const void* src, void* dst, int64_t bytes, hipStream_t st);
hipError_t launch_step64(const snrt_mesh& m, const snrt_quad& q, const StepArgs64& a,
                         const double* psi_in, double* psi_out, const double* S, hipStream_t st);
// the step without scattering through the row-chunked kernel (no in-row reduction); with
// alpha_t = alpha_s = 0 it is the collision-free step of the IMEX splitting
hipError_t launch_free_step32(const snrt_mesh& m, const snrt_quad& q, const StepArgs32& a,
                              const float* psi_in, float* psi_out, hipStream_t st);
hipError_t launch_free_step64(const snrt_mesh& m, const snrt_quad& q, const StepArgs64& a,
                              const double* psi_in, double* psi_out, hipStream_t st);
hipError_t launch_adjoint32(const snrt_mesh& m, const snrt_quad& q, const StepArgs32& a,
                            const float* psi_n, const float* lam_np1, float* lam_n,
                            float* g_t, float* g_s, float* g_r, const float* G, hipStream_t st);
// the FP32 adjoint adding its gradient contributions to FP64 accumulators
hipError_t launch_adjoint32_acc64(const snrt_mesh& m, const snrt_quad& q, const StepArgs32& a,
                                  const float* psi_n, const float* lam_np1, float* lam_n,
                                  double* g_t, double* g_s, double* g_r, const float* G,
                                  hipStream_t st,
                                  const DoseAdj& da = DoseAdj());
hipError_t launch_adjoint64(const snrt_mesh& m, const snrt_quad& q, const StepArgs64& a,
                            const double* psi_n, const double* lam_np1, double* lam_n,
                            double* g_t, double* g_s, double* g_r, const double* G,
                            hipStream_t st);

// Scattering products C[M][N] = A[M][K] X[K][N] (M = ncells).
hipError_t launch_gemm32(const float* A, const float* B, float* C, int64_t M, int32_t K,
                         int32_t N, hipStream_t st);
hipError_t launch_gemm64(const double* A, const double* B, double* C, int64_t M, int32_t K,
                         int32_t N, hipStream_t st);
// What the matrix-core products do with each accumulated element v = (A X)[row][col] (row a
// cell): store it (kStore), or apply the two per-cell steps of the mode-space IMEX solve on
// the way out (IMEX step of Sec. 4.2), with a = 1 + dt alpha_t sigma_t[row] and
// b = dt alpha_s sigma_s[row]:
//   kScale:    C = v * (b / (a - b sig[col]))      the per-cell diagonal on the moments
//   kCombine:  x = C + v, C = x - x y,  y = (a - 1) / a   (C holds the collision-free step)
// Both evaluate exactly the expressions of the separate passes in sn_step_imex.hip.
struct GemmEpi {
    enum : int32_t { kStore = 0, kScale = 1, kCombine = 2 };
    int32_t mode = kStore;
    const float* sigma_t = nullptr;
    const float* sigma_s = nullptr;
    const float* sig = nullptr;
    float dt = 0.0f, alpha_t = 0.0f, alpha_s = 0.0f;
};

// Low-precision products on the matrix cores: X in the hi/lo tiled format with N padded
// columns (N % 128 == 0, K % 32 == 0); C is [M][ldc], ldc <= N.  The FP16 form first writes
// the row exponents of A to rexp [M] (device scratch) and scales X's part by 2^-eb.
hipError_t launch_gemm_bf16(const float* A, const uint16_t* Bhi, const uint16_t* Blo, float* C,
                            int64_t M, int32_t K, int32_t N, int32_t ldc, int products,
                            hipStream_t st, const GemmEpi& epi = GemmEpi());
hipError_t launch_gemm_f16x3(const float* A, const uint16_t* Bhi, const uint16_t* Blo, float* C,
                             int64_t M, int32_t K, int32_t N, int32_t ldc, int32_t* rexp,
                             int32_t eb, hipStream_t st, const GemmEpi& epi = GemmEpi());
// Block shapes of the low-precision products for M rows and N (padded) columns: mbn-wide
// 256-row tiles for the first rows1 rows, tm x tn tiles for the rest (none when rows1 == M).
struct GemmPlan {
    int mbn = 256, tm = 64, tn = 256;
    int64_t rows1 = 0;
};
GemmPlan gemm_plan(int64_t M, int32_t N);
// Row exponents of A [M][K] for the FP16 product into rexp [M] (K % 4 == 0).
hipError_t launch_row_exp_f16(const float* A, int64_t M, int32_t K, int32_t* rexp,
                              hipStream_t st);

// The explicit dense step with the scattering product's last factor and the transport update
// in one launch (sn_step_fused.h): S = A X stays in the product's tiles, each tile updates its
// cells and ordinates from psi_in into psi_out.  A is the product's left operand (psi_in for
// a dense kernel, the moments for the moment form), X its operand in the hi/lo format with
// N = nq columns, N % 256 == 0, K % 32 == 0; triangles only; products as launch_gemm_lp
// (1..3 BF16, 0 FP16 with rexp already written).  The result equals launch_step32's on the
// stored product bit for bit.
// With dpart set, each tile also writes the FP64 sums sum_q w_q psi_in[c][q] (wq: FP64
// weights [nq]) over 128-ordinate pieces of the row: dpart[c * (nq / 128) + piece], for
// k_dose_fold (the fused dose of snrt_step_dose).
struct StepEpi {
    const CellGeom32* geom;
    const float* tab;         // ordinate table [4][nq]
    StepArgs32 a;
    const float* psi_in;
    float* psi_out;
    int64_t nc;
    int32_t nq;
    uint32_t nbf;
    const double* wq;
    double* dpart;
};
// The mode-space IMEX combine in the same one-launch form (the last product of
// snrt_step_imex_dense / _moments): out [nc][nq] holds the collision-free step r and
// receives x - x y, x = r + (A X)[c][q], y = c / (1 + c), c = dt alpha_t sigma_t[c].
struct CombineEpi {
    const float* sigma_t;
    float dt, alpha_t;
    float* out;
    int64_t nc;
    int32_t nq;
};
hipError_t launch_gemm_combine(const float* A, const uint16_t* Bhi, const uint16_t* Blo,
                               int64_t M, int32_t K, int32_t N, int products,
                               const int32_t* rexp, int32_t eb, const CombineEpi& ce,
                               hipStream_t st);

// The transposed dense step in the same one-launch form (snrt_step_adjoint and the reverse
// rollout with a dense or moment-form kernel): the last transposed product's tiles update
// lam_n from lam_np1, psi_n and G = Lambda B^T held in LDS, with the dose functional's term
// (da); the per-cell gradient sums leave as FP32 partial sums over 128-ordinate pieces,
// part[(c * (nq / 128) + piece) * 3 + {t, s, r}], for launch_adjoint_fold.
struct AdjEpi {
    const CellGeom32* geom;
    const float* tab;
    StepArgs32 a;
    const float* psi_n;
    const float* lam_np1;
    float* lam_n;
    int64_t nc;
    int32_t nq;
    float* part;
    DoseAdj da;
};
hipError_t launch_gemm_adjoint(const float* A, const uint16_t* Bhi, const uint16_t* Blo,
                               int64_t M, int32_t K, int32_t N, int products,
                               const int32_t* rexp, int32_t eb, const AdjEpi& ae,
                               hipStream_t st);
// g_t[c] += -dt alpha_t sum_p part_t, g_s[c] += dt alpha_s sum_p part_s,
// g_r[c] += dt (1/rho)^2 sum_p part_r (pieces summed in order in FP32; NULL outputs skipped)
hipError_t launch_adjoint_fold32(int64_t nc, int32_t npieces, const StepArgs32& a,
                                 const float* part, float* g_t, float* g_s, float* g_r,
                                 hipStream_t st);
hipError_t launch_adjoint_fold64(int64_t nc, int32_t npieces, const StepArgs32& a,
                                 const float* part, double* g_t, double* g_s, double* g_r,
                                 hipStream_t st);

namespace fused {
template <bool RHO, bool DOSE>
hipError_t launch_gemm_step_t(const float* A, const uint16_t* Bhi, const uint16_t* Blo,
                              int64_t M, int32_t K, int32_t N, int products,
                              const int32_t* rexp, int32_t eb, const StepEpi& se,
                              hipStream_t st);
// each form is instantiated in a translation unit of its own (sn_step_fused*.hip)
#define SNRT_FUSED_STEP_EXTERN(R, D)                                                          \
    extern template hipError_t launch_gemm_step_t<R, D>(                                      \
        const float*, const uint16_t*, const uint16_t*, int64_t, int32_t, int32_t, int,        \
        const int32_t*, int32_t, const StepEpi&, hipStream_t);
SNRT_FUSED_STEP_EXTERN(false, false)
SNRT_FUSED_STEP_EXTERN(true, false)
SNRT_FUSED_STEP_EXTERN(false, true)
SNRT_FUSED_STEP_EXTERN(true, true)
#undef SNRT_FUSED_STEP_EXTERN
}  // namespace fused
inline hipError_t launch_gemm_step(const float* A, const uint16_t* Bhi, const uint16_t* Blo,
                                   int64_t M, int32_t K, int32_t N, int products,
                                   const int32_t* rexp, int32_t eb, const StepEpi& se,
                                   hipStream_t st) {
    const bool rho = se.a.inv_rho != nullptr, dose = se.dpart != nullptr;
    if (rho)
        return dose ? fused::launch_gemm_step_t<true, true>(A, Bhi, Blo, M, K, N, products,
                                                            rexp, eb, se, st)
                    : fused::launch_gemm_step_t<true, false>(A, Bhi, Blo, M, K, N, products,
                                                             rexp, eb, se, st);
    return dose ? fused::launch_gemm_step_t<false, true>(A, Bhi, Blo, M, K, N, products, rexp,
                                                         eb, se, st)
                : fused::launch_gemm_step_t<false, false>(A, Bhi, Blo, M, K, N, products, rexp,
                                                          eb, se, st);
}

// Re-layout of an FP32 [K][N] matrix (N % 128 == 0) into the BF16 hi/lo operand format of the
// MFMA GEMM, and into the FP16 format of X * 2^eb.
hipError_t launch_split_bf16(const float* B, uint16_t* hi, uint16_t* lo, int32_t K, int32_t N,
                             hipStream_t st);
hipError_t launch_split_f16(const float* B, uint16_t* hi, uint16_t* lo, int32_t K, int32_t N,
                            int32_t eb, hipStream_t st);
// The FP32 product on the matrix cores (K % 32 == 0, N % 128 == 0) and its operand layout.
hipError_t launch_gemm_f32mfma(const float* A, const float* Bt, float* C, int64_t M, int32_t K,
                               int32_t N, hipStream_t st, const GemmEpi& epi = GemmEpi());
hipError_t launch_tile_f32(const float* B, float* out, int32_t K, int32_t N, hipStream_t st);

// IMEX step with the isotropic collision operator taken implicitly (sn_step_imex.hip).
hipError_t launch_imex32(const snrt_mesh& m, const snrt_quad& q, const StepArgs32& a,
                         const float* psi_in, float* psi_out, hipStream_t st);
hipError_t launch_imex64(const snrt_mesh& m, const snrt_quad& q, const StepArgs64& a,
                         const double* psi_in, double* psi_out, hipStream_t st);
// moment-form IMEX: U[c][j] *= b_c / (a_c - b_c Sigma_j), then psi[c][q] = (psi + S) / a_c
hipError_t launch_imex_moment_scale32(const StepArgs32& a, float* U, const float* msig,
                                      int64_t nc, int32_t mid, hipStream_t st);
hipError_t launch_imex_moment_scale64(const StepArgs64& a, double* U, const double* msig,
                                      int64_t nc, int32_t mid, hipStream_t st);
hipError_t launch_imex_combine32(const StepArgs32& a, float* psi, const float* S, int64_t nc,
                                 int32_t nq, hipStream_t st);
hipError_t launch_imex_combine64(const StepArgs64& a, double* psi, const double* S, int64_t nc,
                                 int32_t nq, hipStream_t st);

// Second-order scheme (sn_step2.hip): limited gradient of a stage input and the stage
// update with reconstructed face values; final = true writes (psi_n + stage) / 2.
struct Limiter {
    int32_t kind = SNRT_LIMITER_BARTH_JESPERSEN;
    double k = 0.0;    // Venkatakrishnan's K (eps^2 = (K sqrt(A_i))^3)
};
hipError_t launch_grad2_32(const snrt_mesh& m, const snrt_quad& q, const StepArgs32& a,
                           const Limiter& lim, const float* psi, float* G, hipStream_t st);
hipError_t launch_grad2_64(const snrt_mesh& m, const snrt_quad& q, const StepArgs64& a,
                           const Limiter& lim, const double* psi, double* G, hipStream_t st);
hipError_t launch_flux2_32(const snrt_mesh& m, const snrt_quad& q, const StepArgs32& a,
                           const float* psi, const float* G, const float* S,
                           const float* psi_n, float* out, hipStream_t st);
hipError_t launch_flux2_64(const snrt_mesh& m, const snrt_quad& q, const StepArgs64& a,
                           const double* psi, const double* G, const double* S,
                           const double* psi_n, double* out, hipStream_t st);

hipError_t launch_mass(const snrt_mesh& m, const snrt_quad& q, const float* psi, double* out,
                       hipStream_t st);
hipError_t launch_scalar_flux(const snrt_mesh& m, const snrt_quad& q, const float* psi,
                              float* phi, hipStream_t st);
hipError_t launch_dose(const snrt_mesh& m, const snrt_quad& q, const float* psi,
                       const float* inv_rho, double coeff, double* dose, hipStream_t st);
hipError_t launch_permute(const snrt_mesh& m, int to_user, const void* in, void* out,
                          int64_t row_bytes, hipStream_t st);
hipError_t launch_dose_adjoint(const snrt_mesh& m, const snrt_quad& q, const float* inv_rho,
                               double coeff, const double* g_dose, float* lam, hipStream_t st);
hipError_t launch_dose_density_grad(const snrt_mesh& m, const double* dose, const float* inv_rho,
                                    const double* g_dose, float* g_rho, hipStream_t st);
hipError_t launch_dose_density_grad64(const snrt_mesh& m, const double* dose,
                                      const float* inv_rho, const double* g_dose, double* g_rho,
                                      hipStream_t st);

// P_N step (sn_pn.hip): u_out = step(u_in) in the tiled moment layout; layout conversion
// between the user's [ncells][nm] rows and the tiled internal layout.
// the unrolled FP32 kernel of degree pn::kFusedHighDegree (sn_pn13.hip)
hipError_t launch_pn_fused_high32(const snrt_mesh& m, const snrt_pn& p, const StepArgs32& a,
                                  const float* u, float* out, hipStream_t st);
hipError_t launch_pn32(const snrt_mesh& m, const snrt_pn& p, const StepArgs32& a, const float* u,
                       float* out, hipStream_t st);
hipError_t launch_pn64(const snrt_mesh& m, const snrt_pn& p, const StepArgs64& a, const double* u,
                       double* out, hipStream_t st);
hipError_t launch_pn_layout(const snrt_mesh& m, int32_t nm, int to_user, int elem_bytes,
                            const void* in, void* out, hipStream_t st);
// chunk of output moments per pass of the generic (any degree) P_N kernel
constexpr int kPnChunk32 = 16;
constexpr int kPnChunk64 = 8;

// XCD-aware mapping of a hardware block index to a logical block index: blocks are
// dispatched round-robin over the XCDs, so give XCD x a contiguous range of logical blocks.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
    int64_t x = b % kNumXcd;
    int64_t k = b / kNumXcd;
    int64_t q = nb / kNumXcd, r = nb % kNumXcd;
    return x * q + (x < r ? x : r) + k;
}

}  // namespace snrt
