/*
 * snrt.h -- C ABI of libsnrt, the MI355X (gfx950) explicit S_N step library.
 *
 * The library advances the discrete-ordinates equations of KiT-RT (arXiv 2205.08417)
 *
 *     d_t psi_q + Omega_q . grad(psi_q / rho) + alpha_t Sigma_t psi_q
 *         = alpha_s Sigma_s sum_p w_p k(Omega_q . Omega_p) psi_p + q          (eq. SNEqns,
 *                                                                   eq. BoltzmannCSDTrafo)
 *
 * on an unstructured cell-centred 2-D grid (Sec. 4.1) by one explicit Euler step with the
 * first-order upwind numerical flux (Sec. 4.2, eq. upwind1stOrder2):
 *
 *     psi'_iq = psi_iq - dt/A_i sum_f s_ifq u_up(f,q)
 *               + dt ( -alpha_t sigma_t,i psi_iq + alpha_s sigma_s,i S_iq + q_i ),
 *     s_ifq = Omega_q,x n_if,x + Omega_q,y n_if,y,   u = psi / rho,
 *     u_up = u_i if s_ifq > 0, else the neighbour's u (or the boundary ghost),
 *     S_iq = sum_p K[q][p] w_p psi_ip   (isotropic: K = 1/(4 pi)).
 *
 * Conventions shared by every call:
 *   - Every call returns snrt_status; it never aborts and never throws.  On failure
 *     snrt_last_error() describes the cause (thread-local, valid until the next call on the
 *     same thread).
 *   - Setup calls (snrt_*_create) take HOST FP64 arrays, copy them, and return a handle
 *     owned by the library (free it with the matching *_destroy).  The handle lives on the
 *     HIP device that was current at creation; later calls must run with that device current.
 *   - Per-step calls take DEVICE pointers owned by the caller and a HIP stream (hipStream_t
 *     passed as void*; NULL = the null stream).  They only enqueue work: no host
 *     synchronisation, no allocation.
 *   - psi-like arrays are [ncells][nq] row-major, ordinates fastest, with cells in the
 *     handle's INTERNAL order (a space-filling-curve renumbering chosen at mesh creation;
 *     snrt_permute converts between user and internal order).  Per-cell arrays ([ncells])
 *     are in internal order too.  Boundary-face arrays ([nbfaces][nq]) keep the user's
 *     boundary-face numbering.
 *   - Outputs never alias inputs (SNRT_E_ALIAS).
 *   - Calls that share a handle's internal scratch (snrt_mass) must not overlap in time on
 *     different streams.
 */
#ifndef SNRT_H
#define SNRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SNRT_ABI_VERSION 2

typedef enum {
    SNRT_OK = 0,
    SNRT_E_ARG = -1,          /* null / out-of-range argument */
    SNRT_E_SHAPE = -2,        /* sizes disagree between handles or with the arrays */
    SNRT_E_ALIAS = -3,        /* an output aliases an input */
    SNRT_E_UNSUPPORTED = -4,  /* valid request the library does not implement */
    SNRT_E_HIP = -5,          /* HIP runtime error (text in snrt_last_error) */
    SNRT_E_OOM = -6,          /* device allocation failed */
    SNRT_E_NONFINITE = -7     /* NaN/Inf in a scalar argument */
} snrt_status;

typedef enum {
    SNRT_FP32 = 0,    /* dense scattering product in FP32 (on the matrix cores when the
                         product's inner dimension is a multiple of 32 and its outer one a
                         multiple of 128; FP32 vector FMAs otherwise) */
    SNRT_BF16X3 = 1,  /* BF16 MFMA, hi+lo split of both operands, three products, FP32 accumulate */
    SNRT_BF16X1 = 2,  /* BF16 MFMA, single product (fast, ~1e-3 relative) */
    SNRT_BF16X2 = 3,  /* BF16 MFMA, two products: the scattering operand split hi+lo, the
                         state rounded to BF16 once (its rounding errors are independent
                         across ordinates and average in the sum); FP32 accumulate */
    SNRT_FP16X3 = 4   /* FP16 MFMA, hi+lo split of both operands, three products, FP32
                         accumulate.  FP16 has 11 significant bits but a narrow exponent
                         range, so every state row is scaled by its own power of two (its
                         largest magnitude into [2^13, 2^14)) and the operand by one power of
                         two before the split; the product's rows are scaled back exactly.
                         The row scales come from a pass over the state into the workspace
                         (4 bytes per cell). */
} snrt_precision;

/* mesh flags */
#define SNRT_REORDER_HILBERT 0u  /* renumber cells along a Hilbert curve of the centroids */
#define SNRT_NO_REORDER      1u  /* keep the user's numbering (internal == user order) */

/* boundary treatment of step arguments */
#define SNRT_BC_DIRICHLET 0      /* ghost u = inflow[b][q] * inflow_scale; vacuum if inflow NULL */
#define SNRT_BC_NEUMANN   1      /* ghost u = the cell's own u */

#define SNRT_MAX_NQ 1024         /* ordinates per cell supported by the kernels */

typedef struct snrt_mesh snrt_mesh;
typedef struct snrt_quad snrt_quad;
typedef struct snrt_scatter snrt_scatter;

int snrt_abi_version(void);
const char* snrt_last_error(void);

/* ---------------------------------------------------------------- setup (host FP64 input) */

/* Unstructured grid of Sec. 4.1.  Cell i holds max_faces (3 = triangles, 4 = quadrilaterals)
 * face slots:
 *   face_nbr[i*max_faces+f]         >= 0 neighbour cell (user numbering), -1-b boundary face b
 *                                   (0 <= b < nbfaces), INT32_MIN for an unused slot
 *   face_normal[(i*max_faces+f)*2]  n_ij: outward unit normal times face length
 *   area[i]                         A_i > 0
 *   centroid[i*2]                   used only for the renumbering (may be NULL with
 *                                   SNRT_NO_REORDER)
 * Adjacency must be symmetric.  Returns SNRT_E_ARG for malformed connectivity or areas. */
snrt_status snrt_mesh_create(snrt_mesh** out, int64_t ncells, int32_t max_faces,
                             const int32_t* face_nbr, const double* face_normal,
                             const double* area, const double* centroid, int64_t nbfaces,
                             uint32_t flags);
/* internal_to_user[k] = user index of internal cell k (host array of ncells). */
snrt_status snrt_mesh_permutation(const snrt_mesh* mesh, int64_t* internal_to_user);
snrt_status snrt_mesh_info(const snrt_mesh* mesh, int64_t* ncells, int64_t* nbfaces,
                           int32_t* max_faces);
void snrt_mesh_destroy(snrt_mesh* mesh);

/* Ordinate set (Sec. 3.2): omega[q*3] unit directions (x, y, z), w[q] > 0 weights.
 * 1 <= nq <= SNRT_MAX_NQ.  The streaming uses (x, y); dense kernels use the full vector. */
snrt_status snrt_quad_create(snrt_quad** out, int32_t nq, const double* omega, const double* w);
void snrt_quad_destroy(snrt_quad* quad);

/* Scattering operator S_q = sum_p K[q][p] w_p psi_p of eq. SNEqns.
 * snrt_scatter_isotropic: K = 1/(4 pi) (Sigma_t = Sigma_{s,0} convention of Sec. 2), reduced
 *   per cell without forming K.
 * snrt_scatter_dense: K host [nq*nq] row-major (K[q*nq+p]), applied as a GEMM
 *   S = Psi B with B[p][q] = w_p K[q][p], at the given precision.  The BF16 and FP16 modes
 *   need nq % 32 == 0 (SNRT_E_UNSUPPORTED otherwise); their operand is zero-padded to a
 *   multiple of 128 columns. */
snrt_status snrt_scatter_isotropic(snrt_scatter** out, const snrt_quad* quad);
snrt_status snrt_scatter_dense(snrt_scatter** out, const snrt_quad* quad, const double* K,
                               snrt_precision precision);

/* Moment-projected scattering O Sigma M (eq. SNEqns2): S = O diag(sigma) M psi with the real
 * spherical harmonics m_j of degree <= N = degree ((N+1)^2 moments; Sec. 3.1),
 * O[q][j] = m_j(Omega_q), M[j][q] = w_q m_j(Omega_q), and sigma_l[l] (host, l = 0..N) the
 * kernel's Legendre moments 2 pi int P_l(mu) k(mu) dmu, repeated on the 2l+1 moments of degree
 * l (sigma_0 = 1 conserves particles; Henyey-Greenstein: g^l).  Equivalent to the dense
 * kernel K[q][p] = sum_j m_j(Omega_q) sigma_l(j) m_j(Omega_p), applied as two products through
 * the moments.  0 <= degree <= 30.  The BF16 and FP16 modes need nq % 32 == 0 and pad the
 * moment count with zeros to a multiple of 32.  Steps with this handle need
 * snrt_workspace_size bytes. */
snrt_status snrt_scatter_moments(snrt_scatter** out, const snrt_quad* quad, int32_t degree,
                                 const double* sigma_l, snrt_precision precision);
void snrt_scatter_destroy(snrt_scatter* scatter);

/* Implicit form of a dense kernel, for the IMEX step with dense scattering (Sec. 4.2 with
 * the scattering operator of eq. SNEqns; snrt_step_imex_dense).  Set-up call on a handle
 * from snrt_scatter_dense: decomposes A = K W (A[q][p] = K[q][p] w_p) once, in FP64 on the
 * host, as A = V diag(lam) V^-1 and stores V^-1, V diag(lam) and lam on the device in the
 * handle's precision.  The decomposition goes through the symmetric matrix
 * R^{1/2} A R^{-1/2} for a positive diagonal R with R A symmetric, which exists when K is a
 * symmetric kernel times a positive diagonal (a symmetric kernel with normalised columns,
 * e.g. Henyey-Greenstein; the isotropic kernel as a dense matrix); other kernels return
 * SNRT_E_UNSUPPORTED, as does a decomposition whose residual |A y - V lam V^-1 y| exceeds
 * 1e-10 |A| |y| on seeded probes.  Cost O(nq^3) on one host thread (about a second at
 * nq = 1024), device memory 2 more nq x nq operands.  Idempotent; afterwards
 * snrt_workspace_size includes the implicit solve's workspace.  SNRT_E_UNSUPPORTED for
 * isotropic and moment-form handles. */
snrt_status snrt_scatter_prepare_implicit(snrt_scatter* scatter);

/* The host computation behind snrt_scatter_prepare_implicit, without a device: for
 * A [n][n] (host, row-major, A[q][p] = K[q][p] w_p) it returns the eigenvalues lam [n] and
 * the two operands of the mode-space solve, x0 [n][n] with x0[q][j] = V^-1[j][q] and
 * x1 [n][n] with x1[j][q] = lam_j V[q][j], where A = V diag(lam) V^-1 (all host, FP64,
 * caller-allocated).  resid (may be NULL) receives the probe residual.  Errors as for
 * snrt_scatter_prepare_implicit (SNRT_E_UNSUPPORTED when A is not diagonally similar to a
 * symmetric matrix); SNRT_E_ARG for NULL arrays or n < 1. */
snrt_status snrt_kernel_modes(int32_t n, const double* A, double* lam, double* x0, double* x1,
                              double* resid);

/* Bytes of device workspace that serve every step entry point for this combination:
 * snrt_step / snrt_step_adjoint (FP32 and FP64) need one [ncells][nq] buffer for a dense
 * kernel, plus [ncells][moments, padded] for the moment form, and none for isotropic
 * scattering; snrt_step_dose needs that product buffer (FP32) plus one double per cell and
 * 256-ordinate row chunk of the dense step (one per cell otherwise). */
snrt_status snrt_workspace_size(const snrt_mesh* mesh, const snrt_quad* quad,
                                const snrt_scatter* scatter, size_t* bytes);

/* ---------------------------------------------------------------- per step (device input) */

/* Materials and step scalars.  Device arrays of ncells in internal order unless noted.
 *   sigma_t, sigma_s   required
 *   inv_rho            1/rho (eq. BoltzmannCSDTrafo), NULL means rho = 1
 *   source             isotropic source q_i added as dt*q_i to every ordinate, NULL = 0
 *   inflow             [nbfaces][nq] ghost u = psi/rho on boundary faces (Dirichlet), scaled
 *                      by inflow_scale; NULL = vacuum.  Ignored for SNRT_BC_NEUMANN.
 *   dt                 step; alpha_t, alpha_s multiply sigma_t, sigma_s (1 for time
 *                      problems; energy dependence of CSD cross sections otherwise). */
typedef struct {
    const float* sigma_t;
    const float* sigma_s;
    const float* inv_rho;
    const float* source;
    const float* inflow;
    double inflow_scale;
    double dt;
    double alpha_t;
    double alpha_s;
    int32_t boundary;     /* SNRT_BC_* */
} snrt_step_args;

typedef struct {
    const double* sigma_t;
    const double* sigma_s;
    const double* inv_rho;
    const double* source;
    const double* inflow;
    double inflow_scale;
    double dt;
    double alpha_t;
    double alpha_s;
    int32_t boundary;
} snrt_step_args_f64;

/* One explicit Euler S_N step, FP32: psi_out = step(psi_in).  ws: device workspace of at
 * least snrt_workspace_size bytes (may be NULL for isotropic scattering).  With a dense or
 * moment-form scatter handle in a BF16 / FP16 precision, triangles and nq % 256 == 0 the step
 * runs as one launch: the scattering product's tiles update their cells and ordinates, and
 * S = Psi B never reaches the workspace (the environment variable SNRT_STEP_FUSED=0, read
 * once per process, selects the product-then-step form; both give the same bits). */
snrt_status snrt_step(const snrt_mesh* mesh, const snrt_quad* quad, const snrt_scatter* scatter,
                      const snrt_step_args* args, const float* psi_in, float* psi_out,
                      void* ws, size_t ws_bytes, void* stream);

/* snrt_dose_accumulate(psi_in, args->inv_rho, coeff, dose) followed by snrt_step, with the
 * dose sum taken from the rows the step kernel reads anyway (Sec. 2 pseudo-time dose, left
 * endpoint) instead of a second pass over psi_in:
 *     dose[i] += coeff * inv_rho[i] * sum_q w_q psi_in[i][q]   (FP64; inv_rho NULL = 1)
 * psi_out is bitwise the output of snrt_step; the dose agrees with snrt_dose_accumulate to
 * FP64 rounding (the sum is formed per row piece of the dense step: 128 ordinates in the
 * one-launch form, 256 in the two-launch form; then the pieces are added in order;
 * deterministic).  ws: at least snrt_workspace_size bytes,
 * 16-byte aligned.  dose must not overlap the states or the workspace (SNRT_E_ALIAS);
 * SNRT_E_NONFINITE for a non-finite coeff. */
snrt_status snrt_step_dose(const snrt_mesh* mesh, const snrt_quad* quad,
                           const snrt_scatter* scatter, const snrt_step_args* args,
                           const float* psi_in, float* psi_out, double coeff, double* dose,
                           void* ws, size_t ws_bytes, void* stream);

/* snrt_step_dose for callers that cannot allocate device memory (code under stream capture,
 * serving loops, harnesses that forbid allocation): the same step and dose with isotropic
 * scattering, bitwise the results of snrt_step_dose, but the step's FP64 per-cell dose
 * partials live in a static device array of the library (8 MiB per device, held until the
 * process ends) instead of a workspace.  Needs no workspace and allocates nothing.
 * Limits and errors: at most 1048576 cells (SNRT_E_UNSUPPORTED above); dense and moment
 * scatter handles need the product workspace and are refused (SNRT_E_UNSUPPORTED; use
 * snrt_step_dose); otherwise the errors of snrt_step_dose.  Every call on a device shares
 * that device's array: calls that overlap in time on one device (other streams or threads)
 * race and must be serialised by the caller.  Nothing needs clearing between calls (each
 * call writes every partial it reads). */
snrt_status snrt_step_dose_noalloc(const snrt_mesh* mesh, const snrt_quad* quad,
                                   const snrt_scatter* scatter, const snrt_step_args* args,
                                   const float* psi_in, float* psi_out, double coeff,
                                   double* dose, void* stream);

/* The same step in FP64 throughout (parity template of the FP32 kernels).  Dense scattering
 * runs as an FP64 product regardless of the scatter handle's precision. */
snrt_status snrt_step_f64(const snrt_mesh* mesh, const snrt_quad* quad,
                          const snrt_scatter* scatter, const snrt_step_args_f64* args,
                          const double* psi_in, double* psi_out, void* ws, size_t ws_bytes,
                          void* stream);

/* Adjoint of snrt_step (exact transpose of its linear part, psi' = T psi + b):
 *     lam_n = T^T lam_np1,
 * and the step's gradient contributions, ADDED to each non-NULL output ([ncells], FP32):
 *     g_sigma_t[c] += -dt alpha_t sum_q lam_np1[c][q] psi_n[c][q]
 *     g_sigma_s[c] += dt alpha_s sum_q lam_np1[c][q] S_n[c][q]
 *     g_rho[c]     += sum_q lam_np1 . d psi'/d rho_c   (needs args->inv_rho)
 * psi_n is the state the forward step was applied to.  args->source/inflow do not enter.
 * ws as for snrt_step.  Dense scattering on the conditions of snrt_step's one-launch form
 * (BF16 / FP16 products, triangles, nq a multiple of 256) runs as one launch as well: the
 * transposed product's tiles update lam_n, which is bitwise the two-launch lam_n; each
 * gradient sum then runs over 128-ordinate pieces (in FP32, added in order by a second small
 * kernel) instead of whole rows, so the gradients differ from the two-launch form's in the
 * last bits only.  lam_n must not overlap lam_np1 or psi_n, and with dense scattering the
 * workspace must not overlap psi_n (SNRT_E_ALIAS). */
snrt_status snrt_step_adjoint(const snrt_mesh* mesh, const snrt_quad* quad,
                              const snrt_scatter* scatter, const snrt_step_args* args,
                              const float* psi_n, const float* lam_np1, float* lam_n,
                              float* g_sigma_t, float* g_sigma_s, float* g_rho, void* ws,
                              size_t ws_bytes, void* stream);

/* FP64 adjoint (parity template). */
snrt_status snrt_step_adjoint_f64(const snrt_mesh* mesh, const snrt_quad* quad,
                                  const snrt_scatter* scatter, const snrt_step_args_f64* args,
                                  const double* psi_n, const double* lam_np1, double* lam_n,
                                  double* g_sigma_t, double* g_sigma_s, double* g_rho,
                                  void* ws, size_t ws_bytes, void* stream);

/* The scattering product alone (the S term of eq. SNEqns without the update):
 *   transpose = 0:  S[c][q] = sum_p K[q][p] w_p psi[c][p]          (S = Psi B)
 *   transpose = 1:  S[c][p] = w_p sum_q K[q][p] psi[c][q]          (Lambda B^T, adjoint side)
 * with K the dense kernel, or the kernel of the moment form (eq. SNEqns2).  psi, S: device
 * [ncells][nq] FP32, S must not alias psi.  ws: device workspace of at least
 * snrt_workspace_size bytes, 16-byte aligned and disjoint from psi and S (it holds the
 * moments between the two products of the moment form and the row scales of the FP16 mode;
 * may be NULL for a dense kernel in the FP32 or BF16 modes).  Only for dense and moment
 * scatter handles (SNRT_E_UNSUPPORTED for isotropic). */
snrt_status snrt_scatter_apply(const snrt_mesh* mesh, const snrt_quad* quad,
                               const snrt_scatter* scatter, const float* psi, float* S,
                               int32_t transpose, void* ws, size_t ws_bytes, void* stream);

/* IMEX step (Sec. 4.2): the linear collision operator R psi = -alpha_t sigma_t psi +
 * alpha_s sigma_s S(psi) is taken implicitly, streaming and the source explicitly:
 *     (I - dt R_i) psi_out_i = psi_in_i - dt/A_i sum_f F_up(psi_in) + dt q_i.
 * Isotropic scattering only (SNRT_E_UNSUPPORTED for dense or moment handles; they have
 * snrt_step_imex_dense and snrt_step_imex_moments): the per-cell
 * system has the closed-form solution
 *     psi'_q = (b_q + c B / (a - c W)) / a,  a = 1 + dt alpha_t sigma_t, c = dt alpha_s sigma_s,
 *     B = sum_q w_q b_q / (4 pi),  W = sum_q w_q / (4 pi),
 * which stays positive for any dt sigma (the streaming part keeps its CFL limit).  No
 * workspace. */
snrt_status snrt_step_imex(const snrt_mesh* mesh, const snrt_quad* quad,
                           const snrt_scatter* scatter, const snrt_step_args* args,
                           const float* psi_in, float* psi_out, void* stream);
snrt_status snrt_step_imex_f64(const snrt_mesh* mesh, const snrt_quad* quad,
                               const snrt_scatter* scatter, const snrt_step_args_f64* args,
                               const double* psi_in, double* psi_out, void* stream);

/* IMEX step as above with moment-projected scattering S(psi) = O Sigma M psi (eq. SNEqns2,
 * scatter from snrt_scatter_moments).  Per cell, with a = 1 + dt alpha_t sigma_t and
 * b = dt alpha_s sigma_s, the system (a I - b O Sigma M) psi' = r has, when the quadrature
 * integrates the products of the harmonics exactly (M O = I), the solution
 *     psi' = (r + O D M r) / a,   D = diag(b Sigma_l / (a - b Sigma_l)),
 * computed as the collision-free explicit step r (written to psi_out), the two moment
 * products with the per-cell diagonal between them, and (r + S) / a in place.  Requires
 * a - b Sigma_l != 0 for every moment (always true for sigma_s <= sigma_t, alpha_s <= alpha_t
 * and |Sigma_l| <= 1).  Returns SNRT_E_UNSUPPORTED for other scatter handles and when
 * max |M O - I| > 1e-10 (the product rule integrates degree-N harmonics exactly when it has
 * more than N polar and more than 2N azimuthal nodes; the check is skipped, and the call
 * refused, when (N+1)^4 nq exceeds 2e8).  Workspace: snrt_workspace_size of the handle,
 * 16-byte aligned, disjoint from the states; the products run in the handle's precision. */
snrt_status snrt_step_imex_moments(const snrt_mesh* mesh, const snrt_quad* quad,
                                   const snrt_scatter* scatter, const snrt_step_args* args,
                                   const float* psi_in, float* psi_out, void* workspace,
                                   size_t workspace_bytes, void* stream);
snrt_status snrt_step_imex_moments_f64(const snrt_mesh* mesh, const snrt_quad* quad,
                                       const snrt_scatter* scatter,
                                       const snrt_step_args_f64* args, const double* psi_in,
                                       double* psi_out, void* workspace, size_t workspace_bytes,
                                       void* stream);

/* IMEX step as above with a dense scattering kernel (handle from snrt_scatter_dense, after
 * snrt_scatter_prepare_implicit; SNRT_E_UNSUPPORTED without it).  Per cell, with
 * a = 1 + dt alpha_t sigma_t and b = dt alpha_s sigma_s, the system (a I - b K W) psi' = r
 * has the solution
 *     psi' = (r + V D V^-1 r) / a,   D = diag(b lam_j / (a - b lam_j)),
 * with K W = V diag(lam) V^-1 from the set-up call: the collision-free explicit step r
 * (written to psi_out), the products with V^-1 and V diag(lam) with the per-cell diagonal
 * between them, and (r + S) / a in place.  Requires a - b lam_j != 0 (true for sigma_s <=
 * sigma_t and alpha_s <= alpha_t when the kernel conserves particles, |lam_j| <= 1).
 * Workspace: snrt_workspace_size of the prepared handle (2 nq values per cell, plus one
 * int32 per cell in the FP16 mode), 16-byte aligned, disjoint from the states; the products
 * run in the handle's precision. */
snrt_status snrt_step_imex_dense(const snrt_mesh* mesh, const snrt_quad* quad,
                                 const snrt_scatter* scatter, const snrt_step_args* args,
                                 const float* psi_in, float* psi_out, void* workspace,
                                 size_t workspace_bytes, void* stream);
snrt_status snrt_step_imex_dense_f64(const snrt_mesh* mesh, const snrt_quad* quad,
                                     const snrt_scatter* scatter,
                                     const snrt_step_args_f64* args, const double* psi_in,
                                     double* psi_out, void* workspace, size_t workspace_bytes,
                                     void* stream);

/* ---------------------------------------------------------------- rollouts */

/* Per-step scalars of a multi-step call (the explicit time or energy loop of Alg. "Execution
 * of the solver", one Runge-Kutta stage per step).  HOST arrays of nsteps doubles, each may
 * be NULL (then the value in the step arguments serves every step):
 *   alpha_t, alpha_s, inflow_scale  replace the fields of the same name for step n
 *   dose_coeff                      the dose coefficient of step n (Sec. 2 pseudo-time dose,
 *                                   left endpoint; see snrt_step_dose) */
typedef struct {
    const double* alpha_t;
    const double* alpha_s;
    const double* inflow_scale;
    const double* dose_coeff;
} snrt_schedule;

/* nsteps explicit steps psi^{n+1} = step_n(psi^n), n = 0..nsteps-1, issued from the library on
 * one stream (snrt_step with the step-n arguments; snrt_step_dose when dose is not NULL).
 *   psi    device [ncells][nq]: psi^0 on entry, psi^nsteps on return
 *   tmp    device [ncells][nq] scratch state, disjoint from psi
 *   ckpt   NULL, or device [ceil(nsteps/ckpt_every)][ncells][nq], disjoint from psi and tmp:
 *          on return ckpt[k] holds psi^(k*ckpt_every).  The step before a checkpointed state
 *          writes it into its slot directly (no copies beyond one of psi^0).
 *   dose   NULL, or device [ncells] FP64, accumulated (+=) with sched->dose_coeff[n] before
 *          step n (requires sched->dose_coeff)
 *   ws     as for snrt_step / snrt_step_dose (snrt_workspace_size bytes)
 * States are bitwise those of nsteps separate snrt_step calls.  Errors: those of the step
 * entry points, SNRT_E_ARG (nsteps < 0, ckpt_every < 1 with checkpoints, NULL buffers,
 * dose without dose_coeff), SNRT_E_ALIAS (overlapping buffers).  Host arrays of the
 * schedule are read during the call only; the call returns once every step is enqueued. */
snrt_status snrt_rollout(const snrt_mesh* mesh, const snrt_quad* quad, const snrt_scatter* scatter,
                         const snrt_step_args* args, const snrt_schedule* sched, int64_t nsteps,
                         float* psi, float* tmp, float* ckpt, int32_t ckpt_every, double* dose,
                         void* ws, size_t ws_bytes, void* stream);
snrt_status snrt_rollout_f64(const snrt_mesh* mesh, const snrt_quad* quad,
                             const snrt_scatter* scatter, const snrt_step_args_f64* args,
                             const snrt_schedule* sched, int64_t nsteps, double* psi, double* tmp,
                             double* ckpt, int32_t ckpt_every, void* ws, size_t ws_bytes,
                             void* stream);

/* Reverse pass over a rollout made by snrt_rollout with checkpoints (same args, sched,
 * nsteps and ckpt_every): for each checkpoint segment, last first, the segment's states are
 * recomputed from its checkpoint into seg and walked backwards with the transposed step of
 * snrt_step_adjoint:
 *     lam^N = lam (on entry),  lam^n = T_n^T lam^{n+1} (+ the dose term below),
 * with the gradient contributions of every step added to g_sigma_t, g_sigma_s, g_rho (device
 * [ncells] FP64, accumulated (+=), each may be NULL; g_rho needs args->inv_rho).  The
 * accumulators are FP64 because a long run adds many small contributions of one sign to
 * each cell: an FP32 accumulator loses about half an ulp per addition the same way every
 * time, a drift of order nsteps * 2^-25 relative.
 *   ckpt    device, the checkpoints snrt_rollout wrote
 *   seg     device [ckpt_every - 1][ncells][nq] scratch (may be NULL when ckpt_every == 1)
 *   lam     device [ncells][nq]: dJ/dpsi^N on entry, dJ/dpsi^0 on return
 *   tmp     device [ncells][nq] scratch
 *   g_dose  NULL, or device [ncells] FP64 dJ/dD for a functional of the rollout's dose:
 *           after the transposed step n, snrt_dose_adjoint(args->inv_rho,
 *           sched->dose_coeff[n], g_dose) is applied to lam^n
 *   dose    NULL, or the rollout's dose (device [ncells] FP64): with g_dose and g_rho, the
 *           explicit density derivative -dose_i inv_rho_i g_dose_i is added to g_rho last
 * lam, tmp, seg and ckpt must be disjoint (SNRT_E_ALIAS).  Recomputed states are bitwise the
 * forward ones (the kernels are deterministic), so the result does not depend on ckpt_every. */
snrt_status snrt_rollout_adjoint(const snrt_mesh* mesh, const snrt_quad* quad,
                                 const snrt_scatter* scatter, const snrt_step_args* args,
                                 const snrt_schedule* sched, int64_t nsteps, const float* ckpt,
                                 int32_t ckpt_every, float* seg, float* lam, float* tmp,
                                 double* g_sigma_t, double* g_sigma_s, double* g_rho,
                                 const double* g_dose, const double* dose, void* ws,
                                 size_t ws_bytes, void* stream);
/* The FP64 parity template of the reverse pass (no dose terms). */
snrt_status snrt_rollout_adjoint_f64(const snrt_mesh* mesh, const snrt_quad* quad,
                                     const snrt_scatter* scatter, const snrt_step_args_f64* args,
                                     const snrt_schedule* sched, int64_t nsteps,
                                     const double* ckpt, int32_t ckpt_every, double* seg,
                                     double* lam, double* tmp, double* g_sigma_t,
                                     double* g_sigma_s, double* g_rho, void* ws, size_t ws_bytes,
                                     void* stream);

/* ---------------------------------------------------------------- second-order step */

/* Face-slot midpoints for the second-order scheme (Sec. 4.2, second order finite volume
 * schemes).  face_mid: HOST FP64 [ncells*max_faces*2] in the user's cell order, the
 * midpoint of face slot f of cell c as seen from c (on a periodic mesh, in c's unwrapped
 * frame); entries of unused slots are ignored.  Needs the centroids passed to
 * snrt_mesh_create (SNRT_E_ARG if there were none).  Copied; may be called again to replace
 * them.  Not thread-safe against concurrent steps on the same mesh. */
snrt_status snrt_mesh_set_face_midpoints(snrt_mesh* mesh, const double* face_mid);

/* Bytes of device workspace snrt_step2 (fp64 = 0) or snrt_step2_f64 (fp64 = 1) needs: the
 * intermediate stage state, its limited gradient (two components) and, for dense
 * scattering, the scattering product -- each [ncells][nq] of the step's element type. */
snrt_status snrt_step2_workspace_size(const snrt_mesh* mesh, const snrt_quad* quad,
                                      const snrt_scatter* scatter, int32_t fp64, size_t* bytes);

/* One step of the second-order scheme: the Heun method
 *     psi* = L(psi_in),  psi** = L(psi*),  psi_out = (psi_in + psi**) / 2,
 * where L is the explicit Euler update above with the upwind flux fed by limited linear
 * reconstructions of u = psi/rho on both sides of every face,
 *     u~_i = u_i + Psi_i grad(u_i) . r_if,   r_if = face midpoint - centroid_i,
 * grad(u_i) the Green-Gauss gradient from face averages (u_i + u_j)/2 (boundary faces use
 * the ghost value) and Psi_i the Barth-Jespersen limiter (snrt_step2_limited below offers
 * Venkatakrishnan's as well) with the extremes of u over the
 * cell and its face neighbours and the increment grad(u_i) . r_if.  Ghost values are not
 * reconstructed.  Both stages use args (the same alpha_t, alpha_s, inflow_scale).
 * Requires snrt_mesh_set_face_midpoints (SNRT_E_ARG otherwise) and a workspace of
 * snrt_step2_workspace_size bytes; psi_out must not alias psi_in or the workspace. */
snrt_status snrt_step2(const snrt_mesh* mesh, const snrt_quad* quad, const snrt_scatter* scatter,
                       const snrt_step_args* args, const float* psi_in, float* psi_out,
                       void* ws, size_t ws_bytes, void* stream);

/* The second-order step in FP64 throughout (parity template). */
snrt_status snrt_step2_f64(const snrt_mesh* mesh, const snrt_quad* quad,
                           const snrt_scatter* scatter, const snrt_step_args_f64* args,
                           const double* psi_in, double* psi_out, void* ws, size_t ws_bytes,
                           void* stream);

/* Slope limiter of the second-order step (Sec. 4.2 names Barth-Jespersen and
 * Venkatakrishnan).  With d = grad(u_i) . r_if the unlimited increment at face f and
 * d1 = u_max - u_i (d > 0) or u_min - u_i (d < 0), both limiters scale the gradient by
 * Psi_i = min over the faces of phi(d1, d), phi = 1 where d = 0:
 *   SNRT_LIMITER_BARTH_JESPERSEN:  phi = min(1, d1 / d)
 *   SNRT_LIMITER_VENKATAKRISHNAN:  phi = (d1^2 + eps^2 + 2 d d1) / (d1^2 + 2 d^2 + d d1 + eps^2),
 *                                  eps^2 = (k sqrt(A_i))^3
 * The Venkatakrishnan form is smooth in the data.  With k = 0 it keeps every reconstructed
 * value inside the neighbourhood range (phi <= d1 / d) though phi itself may exceed 1
 * slightly; a larger k limits less wherever the variation is small against eps. */
#define SNRT_LIMITER_BARTH_JESPERSEN 0
#define SNRT_LIMITER_VENKATAKRISHNAN 1
typedef struct snrt_limiter {
    int32_t kind;       /* SNRT_LIMITER_* */
    int32_t reserved;   /* 0 */
    double k;           /* Venkatakrishnan's K >= 0 (length-scale factor); ignored otherwise */
} snrt_limiter;

/* snrt_step2 / snrt_step2_f64 with the limiter chosen by lim (NULL = Barth-Jespersen, which
 * is what snrt_step2 uses).  SNRT_E_ARG for an unknown kind, a non-zero reserved field or a
 * k that is negative or not finite; everything else as snrt_step2. */
snrt_status snrt_step2_limited(const snrt_mesh* mesh, const snrt_quad* quad,
                               const snrt_scatter* scatter, const snrt_step_args* args,
                               const snrt_limiter* lim, const float* psi_in, float* psi_out,
                               void* ws, size_t ws_bytes, void* stream);
snrt_status snrt_step2_limited_f64(const snrt_mesh* mesh, const snrt_quad* quad,
                                   const snrt_scatter* scatter, const snrt_step_args_f64* args,
                                   const snrt_limiter* lim, const double* psi_in,
                                   double* psi_out, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- reductions */

/* Total mass sum_i A_i sum_q w_q psi_iq accumulated in FP64 (solver log, Sec. 5.1), written
 * to out_dev (one device double).  Deterministic two-pass tree. */
snrt_status snrt_mass(const snrt_mesh* mesh, const snrt_quad* quad, const float* psi,
                      double* out_dev, void* stream);

/* Scalar flux phi_i = sum_q w_q psi_iq (Sec. 7.2), FP64 accumulation rounded to FP32. */
snrt_status snrt_scalar_flux(const snrt_mesh* mesh, const snrt_quad* quad, const float* psi,
                             float* phi, void* stream);

/* Dose term (Sec. 2, integral in pseudo-time, left endpoint):
 *     dose[i] += coeff * inv_rho[i] * sum_q w_q psi_iq      (FP64, inv_rho NULL = 1). */
snrt_status snrt_dose_accumulate(const snrt_mesh* mesh, const snrt_quad* quad, const float* psi,
                                 const float* inv_rho, double coeff, double* dose,
                                 void* stream);

/* Adjoint of snrt_dose_accumulate for a functional J(D): with g_dose = dJ/dD,
 *     lam[i][q] += coeff * w_q * inv_rho[i] * g_dose[i]          (lam FP32, g_dose FP64)
 * (the dose term of step n contributes coeff_n w_q (dJ/dD_i) / rho_i to dJ/dpsi^n_iq). */
snrt_status snrt_dose_adjoint(const snrt_mesh* mesh, const snrt_quad* quad, const float* inv_rho,
                              double coeff, const double* g_dose, float* lam, void* stream);

/* Explicit density derivative of the dose D_i = (1/rho_i) sum_n coeff_n phi_i^n:
 *     g_rho[i] += -dose[i] * inv_rho[i] * g_dose[i]             (g_rho FP32, dose/g_dose FP64) */
snrt_status snrt_dose_density_grad(const snrt_mesh* mesh, const double* dose,
                                   const float* inv_rho, const double* g_dose, float* g_rho,
                                   void* stream);

/* ---------------------------------------------------------------- P_N solver (Sec. 4.3) */

/* The P_N moment system of degree N (Sec. 3.1, P_N closure): the state of a cell is the
 * vector u of the (N+1)^2 moments u_j = int psi m_j dOmega with the real spherical harmonics
 * m_j, j = l^2 + l + k (the ordering of snrt_scatter_moments), and
 *     d_t u + A_x d_x (u/rho) + A_y d_y (u/rho) + alpha_t sigma_t u
 *         = alpha_s sigma_s Sigma u + sqrt(4 pi) q e_0,
 *     A_x = int m m^T Omega_x dOmega,  A_y = int m m^T Omega_y dOmega,
 *     Sigma = diag(sigma_l(j)) (the kernel's Legendre moments on every moment of degree l).
 * One explicit Euler step uses the upwind flux of Sec. 4.3 with the Jacobians split into
 * their positive and negative semidefinite parts A = A^+ + A^- (eigen-decomposition):
 *     F(u_i, u_j) = sum_{l=x,y} n_l (A_l^+ u_i/rho_i + A_l^- u_j/rho_j)   if n_l > 0,
 *                               n_l (A_l^- u_i/rho_i + A_l^+ u_j/rho_j)   otherwise,
 *     u_i' = u_i - dt/A_i sum_f F + dt (-alpha_t sigma_t u_i + alpha_s sigma_s Sigma u_i
 *                                        + sqrt(4 pi) q_i e_0).
 * The kernels evaluate the algebraically identical per-cell form
 * (A_x X + A_y Y + |A_x| P + |A_y| Q) / 2 with |A| = A^+ - A^- and X, Y, P, Q sums over the
 * faces of n (u_i/rho_i + u_j/rho_j) and |n| (u_i/rho_i - u_j/rho_j); results agree with the
 * face-by-face formula up to rounding. */
typedef struct snrt_pn snrt_pn;

/* Host-only: the library's A_x, A_y, |A_x| = A_x^+ - A_x^-, |A_y| for degree N (each
 * [(N+1)^2][(N+1)^2] row-major FP64, any pointer may be NULL).  No device is used.
 * 0 <= degree <= 30. */
snrt_status snrt_pn_operators(int32_t degree, double* ax, double* ay, double* ax_abs,
                              double* ay_abs);

/* P_N system of the given degree (0..30) on the current device.  sigma_l: host [degree+1]
 * Legendre moments of the scattering kernel (2 pi int P_l(mu) k(mu) dmu; sigma_0 = 1
 * conserves particles), NULL = isotropic (1, 0, 0, ...).  Degrees up to 9 run a fully
 * unrolled kernel; larger degrees a chunked one. */
snrt_status snrt_pn_create(snrt_pn** out, int32_t degree, const double* sigma_l);
void snrt_pn_destroy(snrt_pn* pn);
snrt_status snrt_pn_info(const snrt_pn* pn, int32_t* degree, int32_t* nmoments);

/* Elements of a P_N state array: the tiled layout below, ceil(ncells/64)*64*nmoments. */
snrt_status snrt_pn_state_elems(const snrt_mesh* mesh, const snrt_pn* pn, int64_t* elems);

/* P_N state layout.  Cells in the mesh's internal order, grouped in tiles of 64 cells,
 * moment-major inside a tile: element (internal cell c, moment j) is at
 * ((c / 64) * nmoments + j) * 64 + c % 64.  Padding cells of the last tile are never read.
 * snrt_pn_layout converts device arrays between the user's [ncells][nmoments] rows in user
 * cell order (to_user = 0: user -> tiled; 1: tiled -> user), elem_bytes 4 (FP32) or 8. */
snrt_status snrt_pn_layout(const snrt_mesh* mesh, const snrt_pn* pn, int32_t to_user,
                           int32_t elem_bytes, const void* in, void* out, void* stream);

/* One explicit Euler P_N step, u_out = step(u_in), both device arrays in the tiled layout,
 * 16-byte aligned, not aliased.  args as for snrt_step, with two differences: source is the
 * isotropic q_i (entering moment 0 as sqrt(4 pi) dt q_i) and inflow holds ghost MOMENTS
 * [nbfaces][nmoments] in u/rho units (scaled by inflow_scale; NULL = vacuum; Neumann uses
 * the cell's own u/rho).  No workspace. */
snrt_status snrt_pn_step(const snrt_mesh* mesh, const snrt_pn* pn, const snrt_step_args* args,
                         const float* u_in, float* u_out, void* stream);
snrt_status snrt_pn_step_f64(const snrt_mesh* mesh, const snrt_pn* pn,
                             const snrt_step_args_f64* args, const double* u_in, double* u_out,
                             void* stream);

/* Row permutation between user (direction 0 -> internal) and internal (direction 1 -> user)
 * cell order for [ncells][row_bytes] device arrays; row_bytes a positive multiple of 4. */
snrt_status snrt_permute(const snrt_mesh* mesh, int32_t to_user, const void* in, void* out,
                         int64_t row_bytes, void* stream);

/* ---------------------------------------------------------------- measurement helper */

/* Not part of the method: copies `bytes` bytes from src to dst (device pointers, 16-byte
 * aligned, disjoint; bytes a non-negative multiple of 16) in one launch on `stream`, with
 * 16-byte nontemporal loads and stores.  Its rate on a state-sized buffer is the attainable
 * HBM read+write bandwidth that the step kernels are compared with.  SNRT_E_ARG for a bad
 * size, a NULL or misaligned pointer (bytes > 0); SNRT_E_ALIAS if the ranges overlap. */
snrt_status snrt_stream_copy(const void* src, void* dst, int64_t bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SNRT_H */
