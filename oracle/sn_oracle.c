/*
 * sn_oracle.c -- plain FP64 CPU reference of the explicit S_N step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links or calls this file: it is
 * used by tests/, by smoke() in __graft_entry__.py and by the CPU-baseline leg of
 * bench.py.  It shares no code, header or constant with the HIP library.
 *
 * What it computes (KiT-RT, arXiv 2205.08417):
 *   S_N equations with density (eq. SNEqns, eq. BoltzmannCSDTrafo)
 *       d_t psi_q + Omega_q . grad(psi_q / rho) + Sigma_t psi_q = sum_p w_p Sigma_s(Omega_q.Omega_p) psi_p (+ q)
 *   discretised with the cell-centred finite-volume scheme of Sec. 4.2: first-order upwind
 *   numerical flux (eq. upwind1stOrder, specialised to S_N in eq. upwind1stOrder2) and the
 *   explicit Euler update
 *       psi_i^{n+1} = psi_i^n - dt/A_i sum_{j in N(i)} F_up(psi_j, psi_i) + dt R(psi_i^n).
 *   Cells carry n_{i,j} = outward unit normal times face length (Sec. 4.1).
 *
 * Readings where the paper leaves freedom (all listed in the design notes):
 *   - H(x) = 1 for x > 0 and 0 otherwise: a face with Omega.n = 0 takes the neighbour branch,
 *     whose contribution is 0 * u either way.
 *   - isotropic scattering is the kernel 1/(4 pi) (Sigma_t = Sigma_{s,0}, Sec. 2).
 *   - the source q_i is an angular density added as dt*q_i to every ordinate.
 *   - per-step multipliers alpha_t, alpha_s scale Sigma_t and Sigma_s (energy dependence of
 *     the CSD cross sections, eq. BoltzmannCSDTrafo); 1 for time-dependent problems.
 *   - boundary faces take a ghost value of u = psi/rho: inflow[b*nq+q]*inflow_scale
 *     (Dirichlet; vacuum when inflow is NULL), or the cell's own u (Neumann).
 *
 * Array conventions (all host memory, caller-owned, row-major):
 *   face_nbr[c*mf+f]        >= 0 neighbour, -1-b boundary face b, INT32_MIN unused slot
 *   face_normal[(c*mf+f)*2] outward normal times length
 *   omega[q*3]              unit direction (x, y, z); streaming uses (x, y)
 *   K[q*nq+p]               dense kernel: S_q = sum_p K[q][p] w_p psi_p; NULL = isotropic
 *   psi[c*nq+q]
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_UNUSED_FACE INT32_MIN

static const double oracle_pi = 3.14159265358979323846264338327950288;

int oracle_version(void) { return 1; }

#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads a parallel region of this library uses (reported beside CPU timings). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the thread count of the following parallel loops (n >= 1); returns the previous one. */
int oracle_set_num_threads(int n)
{
    int prev = oracle_num_threads();
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
    return prev;
}

/* Scattering source of cell c at ordinate q: sum_p k(Omega_q.Omega_p) w_p psi_cp (eq. SNEqns). */
static double scatter_source(int32_t nq, const double* w, const double* K, const double* psi_c, int32_t q)
{
    double s = 0.0;
    if (K == NULL) {
        for (int32_t p = 0; p < nq; ++p) s += w[p] * psi_c[p];
        return s / (4.0 * oracle_pi);
    }
    for (int32_t p = 0; p < nq; ++p) s += K[(size_t)q * nq + p] * w[p] * psi_c[p];
    return s;
}

/* One explicit Euler step.  With sel != NULL only cells sel[0..nsel) are computed and row k
 * of psi_out belongs to cell sel[k]; otherwise psi_out is [nc][nq]. */
int oracle_step(int64_t nc, int32_t mf, const int32_t* face_nbr, const double* face_normal,
                const double* area, int32_t nq, const double* omega, const double* w,
                const double* K, const double* sigma_t, const double* sigma_s, const double* rho,
                const double* source, const double* inflow, double inflow_scale, int32_t neumann,
                double dt, double alpha_t, double alpha_s, const double* psi_in, double* psi_out,
                int64_t nsel, const int64_t* sel)
{
    if (nc < 0 || mf < 1 || nq < 1 || !face_nbr || !face_normal || !area || !omega || !w ||
        !sigma_t || !sigma_s || !psi_in || !psi_out)
        return -1;
    int64_t count = sel ? nsel : nc;
    int failed = 0;
#pragma omp parallel
    {
        /* scattering source of the current cell, all ordinates (eq. SNEqns) */
        double* S = (double*)malloc(sizeof(double) * (size_t)nq);
        if (!S) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(static)
        for (int64_t k = 0; k < count; ++k) {
            if (!S) continue;
            int64_t i = sel ? sel[k] : k;
            const double* psi_i = psi_in + (size_t)i * nq;
            double rho_i = rho ? rho[i] : 1.0;
            double* out = psi_out + (size_t)k * nq;
            if (K == NULL) {
                double iso = scatter_source(nq, w, NULL, psi_i, 0);
                for (int32_t q = 0; q < nq; ++q) S[q] = iso;
            } else {
                for (int32_t q = 0; q < nq; ++q) S[q] = scatter_source(nq, w, K, psi_i, q);
            }
            for (int32_t q = 0; q < nq; ++q) {
                /* numerical flux sum over the faces of cell i (eq. upwind1stOrder2) */
                double flux = 0.0;
                for (int32_t f = 0; f < mf; ++f) {
                    int32_t j = face_nbr[(size_t)i * mf + f];
                    if (j == ORACLE_UNUSED_FACE) continue;
                    const double* n = face_normal + ((size_t)i * mf + f) * 2;
                    double s = omega[(size_t)q * 3 + 0] * n[0] + omega[(size_t)q * 3 + 1] * n[1];
                    double u_i = psi_i[q] / rho_i;
                    double u_j;
                    if (j >= 0) {
                        u_j = psi_in[(size_t)j * nq + q] / (rho ? rho[j] : 1.0);
                    } else if (neumann) {
                        u_j = u_i;
                    } else {
                        int64_t b = -1 - (int64_t)j;
                        u_j = inflow ? inflow[(size_t)b * nq + q] * inflow_scale : 0.0;
                    }
                    double H = s > 0.0 ? 1.0 : 0.0;
                    flux += s * u_i * H + s * u_j * (1.0 - H);
                }
                /* right-hand side: absorption/total, scattering, source */
                double R = -alpha_t * sigma_t[i] * psi_i[q] + alpha_s * sigma_s[i] * S[q]
                           + (source ? source[i] : 0.0);
                out[q] = psi_i[q] - dt / area[i] * flux + dt * R;
            }
        }
        free(S);
    }
    if (failed) return -2;
    return 0;
}

/* Transposed step: lam_n = T^T lam_np1, where psi^{n+1} = T psi^n + b is the step above.
 * The transpose is formed by walking the forward step's coefficients and scattering each
 * one, multiplied by lam_np1 at the output entry, into the input entry it came from.
 * Gradient contributions of this step are ADDED to g_sigma_t, g_sigma_s, g_rho (each may be
 * NULL):  sum_{i,q} lam_np1[i][q] * d psi^{n+1}[i][q] / d theta  at psi = psi_n. */
int oracle_adjoint_step(int64_t nc, int32_t mf, const int32_t* face_nbr, const double* face_normal,
                        const double* area, int32_t nq, const double* omega, const double* w,
                        const double* K, const double* sigma_t, const double* sigma_s,
                        const double* rho, int32_t neumann, double dt, double alpha_t,
                        double alpha_s, const double* psi_n, const double* lam_np1, double* lam_n,
                        double* g_sigma_t, double* g_sigma_s, double* g_rho)
{
    if (nc < 0 || mf < 1 || nq < 1 || !face_nbr || !face_normal || !area || !omega || !w ||
        !sigma_t || !sigma_s || !psi_n || !lam_np1 || !lam_n)
        return -1;
    memset(lam_n, 0, sizeof(double) * (size_t)nc * nq);

    /* streaming: each coefficient couples the same ordinate q, so ordinates are independent */
#pragma omp parallel for schedule(static)
    for (int32_t q = 0; q < nq; ++q) {
        for (int64_t i = 0; i < nc; ++i) {
            double l = lam_np1[(size_t)i * nq + q];
            for (int32_t f = 0; f < mf; ++f) {
                int32_t j = face_nbr[(size_t)i * mf + f];
                if (j == ORACLE_UNUSED_FACE) continue;
                const double* n = face_normal + ((size_t)i * mf + f) * 2;
                double s = omega[(size_t)q * 3 + 0] * n[0] + omega[(size_t)q * 3 + 1] * n[1];
                double a = -dt / area[i] * s;  /* coefficient of the upwind u in psi^{n+1}_iq */
                int64_t up;
                if (s > 0.0) up = i;
                else if (j >= 0) up = j;
                else if (neumann) up = i;
                else continue;                   /* Dirichlet ghost: affine part b */
                double rho_up = rho ? rho[up] : 1.0;
                lam_n[(size_t)up * nq + q] += a / rho_up * l;
            }
        }
    }
    /* gradient w.r.t. rho: d(psi_up/rho_up)/d rho_up = -psi_up/rho_up^2 */
    if (g_rho && rho) {
        for (int64_t i = 0; i < nc; ++i) {
            for (int32_t q = 0; q < nq; ++q) {
                double l = lam_np1[(size_t)i * nq + q];
                for (int32_t f = 0; f < mf; ++f) {
                    int32_t j = face_nbr[(size_t)i * mf + f];
                    if (j == ORACLE_UNUSED_FACE) continue;
                    const double* n = face_normal + ((size_t)i * mf + f) * 2;
                    double s = omega[(size_t)q * 3 + 0] * n[0] + omega[(size_t)q * 3 + 1] * n[1];
                    double a = -dt / area[i] * s;
                    int64_t up;
                    if (s > 0.0) up = i;
                    else if (j >= 0) up = j;
                    else if (neumann) up = i;
                    else continue;
                    double r = rho[up];
                    g_rho[up] += a * (-psi_n[(size_t)up * nq + q] / (r * r)) * l;
                }
            }
        }
    }
    /* local terms: identity, total cross section, scattering (couples ordinates of one cell) */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nc; ++i) {
        const double* l = lam_np1 + (size_t)i * nq;
        const double* psi_i = psi_n + (size_t)i * nq;
        double* out = lam_n + (size_t)i * nq;
        double gt = 0.0, gs = 0.0;
        double iso = K ? 0.0 : scatter_source(nq, w, NULL, psi_i, 0);
        for (int32_t q = 0; q < nq; ++q) {
            out[q] += (1.0 - dt * alpha_t * sigma_t[i]) * l[q];
            double c = dt * alpha_s * sigma_s[i];
            for (int32_t p = 0; p < nq; ++p) {
                double kqp = K ? K[(size_t)q * nq + p] : 1.0 / (4.0 * oracle_pi);
                out[p] += c * kqp * w[p] * l[q];
            }
            gt += -dt * alpha_t * psi_i[q] * l[q];
            double S_q = K ? scatter_source(nq, w, K, psi_i, q) : iso;
            gs += dt * alpha_s * S_q * l[q];
        }
        if (g_sigma_t) g_sigma_t[i] += gt;
        if (g_sigma_s) g_sigma_s[i] += gs;
    }
    return 0;
}

/* Total mass sum_i A_i sum_q w_q psi_iq (the quantity the solver log reports, Sec. 5.1). */
double oracle_mass(int64_t nc, const double* area, int32_t nq, const double* w, const double* psi)
{
    double m = 0.0;
    for (int64_t i = 0; i < nc; ++i) {
        double phi = 0.0;
        for (int32_t q = 0; q < nq; ++q) phi += w[q] * psi[(size_t)i * nq + q];
        m += area[i] * phi;
    }
    return m;
}

/* Scalar flux Psi_i = sum_q w_q psi_iq (quadrature of int_{S^2} psi dOmega, Sec. 7.2). */
int oracle_scalar_flux(int64_t nc, int32_t nq, const double* w, const double* psi, double* phi)
{
    if (!w || !psi || !phi) return -1;
    for (int64_t i = 0; i < nc; ++i) {
        double s = 0.0;
        for (int32_t q = 0; q < nq; ++q) s += w[q] * psi[(size_t)i * nq + q];
        phi[i] = s;
    }
    return 0;
}

/* One left-endpoint term of the dose integral of Sec. 2 in pseudo-time:
 *   D_i += coeff / rho_i * sum_q w_q psi_iq,  coeff = dt_n * S(E_n). */
int oracle_dose_accumulate(int64_t nc, int32_t nq, const double* w, const double* psi,
                           const double* rho, double coeff, double* dose)
{
    if (!w || !psi || !dose) return -1;
    for (int64_t i = 0; i < nc; ++i) {
        double s = 0.0;
        for (int32_t q = 0; q < nq; ++q) s += w[q] * psi[(size_t)i * nq + q];
        dose[i] += coeff / (rho ? rho[i] : 1.0) * s;
    }
    return 0;
}

/* ---------------------------------------------------------------------------------------
 * Second-order scheme (Sec. 4.2, second order finite volume schemes): the flux inputs are
 * linear reconstructions u_i + Psi_i grad(u_i) . r_ij with a Green-Gauss gradient built
 * from face averages and the Barth-Jespersen limiter Psi_i, and time advances with the
 * two-stage Heun scheme  psi* = L(psi^n), psi** = L(psi*), psi^{n+1} = (psi^n + psi**)/2,
 * where L is one explicit Euler stage with the reconstructed upwind flux.
 *
 * Readings (listed in the design notes):
 *   - the reconstructed variable is u = psi/rho, the quantity the upwind flux transports;
 *   - the limiter's increment is the one the reconstruction adds, Delta_2 = grad u_i . r_ij
 *     (the printed factor 1/2 contradicts the reconstruction the limiter is meant to bound);
 *   - g_max and g_min are the extremes of u over the cell and every value across its faces,
 *     the definition of the cited Barth-Jespersen limiter.  Taken face by face, as the
 *     printed formula can be read, the limiter clips smooth data so often that the scheme
 *     is only first order (measured), against the section's claim of second order;
 *   - a boundary face's u_j is the first-order ghost value; it enters the Green-Gauss sum
 *     and the limiter like a neighbour value and is not itself reconstructed;
 *   - both Heun stages use the step's alpha_t, alpha_s and inflow scale and add dt*R (the
 *     first-order update's source term), not dt/A_i*R.
 * Extra arrays: face_mid[(c*mf+f)*2] is the midpoint of face slot f as seen from cell c (on
 * a periodic mesh, in c's unwrapped frame) and centroid[c*2] the cell centroid.
 * --------------------------------------------------------------------------------------- */

/* u on the far side of face f of cell i at ordinate q: neighbour value or ghost value */
static double far_u(int64_t i, int32_t mf, const int32_t* face_nbr, int32_t f, int32_t nq,
                    int32_t q, const double* rho, const double* inflow, double inflow_scale,
                    int32_t neumann, const double* psi)
{
    int32_t j = face_nbr[(size_t)i * mf + f];
    double u_i = psi[(size_t)i * nq + q] / (rho ? rho[i] : 1.0);
    if (j >= 0) return psi[(size_t)j * nq + q] / (rho ? rho[j] : 1.0);
    if (neumann) return u_i;
    int64_t b = -1 - (int64_t)j;
    return inflow ? inflow[(size_t)b * nq + q] * inflow_scale : 0.0;
}

/* Limited gradient Psi_i grad(u_i) of every cell and ordinate into gx, gy [nc][nq]. */
/* limiter: 0 = Barth-Jespersen; 1 = Venkatakrishnan with eps^2 = (vk_k sqrt(A_i))^3 */
int oracle_limited_gradient(int64_t nc, int32_t mf, const int32_t* face_nbr,
                            const double* face_normal, const double* face_mid,
                            const double* centroid, const double* area, int32_t nq,
                            const double* rho, const double* inflow, double inflow_scale,
                            int32_t neumann, int32_t limiter, double vk_k, const double* psi,
                            double* gx, double* gy)
{
    if (nc < 0 || mf < 1 || nq < 1 || !face_nbr || !face_normal || !face_mid || !centroid ||
        !area || !psi || !gx || !gy || (limiter != 0 && limiter != 1))
        return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nc; ++i) {
        double rho_i = rho ? rho[i] : 1.0;
        for (int32_t q = 0; q < nq; ++q) {
            double u_i = psi[(size_t)i * nq + q] / rho_i;
            /* Green-Gauss with the face value (u_i + u_j)/2 */
            double ax = 0.0, ay = 0.0;
            for (int32_t f = 0; f < mf; ++f) {
                if (face_nbr[(size_t)i * mf + f] == ORACLE_UNUSED_FACE) continue;
                const double* n = face_normal + ((size_t)i * mf + f) * 2;
                double u_j = far_u(i, mf, face_nbr, f, nq, q, rho, inflow, inflow_scale,
                                   neumann, psi);
                ax += 0.5 * (u_i + u_j) * n[0];
                ay += 0.5 * (u_i + u_j) * n[1];
            }
            ax /= area[i];
            ay /= area[i];
            /* extremes of u over the cell and all the values across its faces */
            double gmax = u_i, gmin = u_i;
            for (int32_t f = 0; f < mf; ++f) {
                if (face_nbr[(size_t)i * mf + f] == ORACLE_UNUSED_FACE) continue;
                double u_j = far_u(i, mf, face_nbr, f, nq, q, rho, inflow, inflow_scale,
                                   neumann, psi);
                if (u_j > gmax) gmax = u_j;
                if (u_j < gmin) gmin = u_j;
            }
            /* the smallest scaling over the faces: Barth-Jespersen admits at most 1 and the
               increment up to the extreme; Venkatakrishnan replaces min(1, d1/d2) by a
               smooth function of d1/d2 with the threshold eps^2 */
            double eps2 = 0.0;
            if (limiter == 1) {
                double h = vk_k * sqrt(area[i]);
                eps2 = h * h * h;
            }
            double lim = 1.0;
            for (int32_t f = 0; f < mf; ++f) {
                if (face_nbr[(size_t)i * mf + f] == ORACLE_UNUSED_FACE) continue;
                const double* m = face_mid + ((size_t)i * mf + f) * 2;
                double rx = m[0] - centroid[(size_t)i * 2 + 0];
                double ry = m[1] - centroid[(size_t)i * 2 + 1];
                double d2 = ax * rx + ay * ry;
                double t = 1.0;
                if (d2 != 0.0) {
                    double d1 = d2 > 0.0 ? gmax - u_i : gmin - u_i;
                    if (limiter == 1) {
                        t = ((d1 * d1 + eps2) * d2 + 2.0 * d2 * d2 * d1) /
                            (d1 * d1 + 2.0 * d2 * d2 + d1 * d2 + eps2) / d2;
                    } else {
                        t = d1 / d2;
                        if (t > 1.0) t = 1.0;
                    }
                }
                if (t < lim) lim = t;
            }
            gx[(size_t)i * nq + q] = lim * ax;
            gy[(size_t)i * nq + q] = lim * ay;
        }
    }
    return 0;
}

/* Slot of cell j whose neighbour is cell i (the shared face seen from j), or -1. */
static int32_t back_slot(int64_t j, int64_t i, int32_t mf, const int32_t* face_nbr)
{
    for (int32_t f = 0; f < mf; ++f)
        if (face_nbr[(size_t)j * mf + f] == (int32_t)i) return f;
    return -1;
}

/* One explicit Euler stage with the reconstructed upwind flux: out = psi - dt/A sum F + dt R. */
static int stage2(int64_t nc, int32_t mf, const int32_t* face_nbr, const double* face_normal,
                  const double* face_mid, const double* centroid, const double* area, int32_t nq,
                  const double* omega, const double* w, const double* K, const double* sigma_t,
                  const double* sigma_s, const double* rho, const double* source,
                  const double* inflow, double inflow_scale, int32_t neumann, double dt,
                  double alpha_t, double alpha_s, int32_t limiter, double vk_k, const double* psi,
                  double* out, double* gx, double* gy)
{
    int rc = oracle_limited_gradient(nc, mf, face_nbr, face_normal, face_mid, centroid, area, nq,
                                     rho, inflow, inflow_scale, neumann, limiter, vk_k, psi, gx,
                                     gy);
    if (rc != 0) return rc;
    int failed = 0;
#pragma omp parallel
    {
        double* S = (double*)malloc(sizeof(double) * (size_t)nq);
        if (!S) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(static)
        for (int64_t i = 0; i < nc; ++i) {
            if (!S) continue;
            const double* psi_i = psi + (size_t)i * nq;
            double rho_i = rho ? rho[i] : 1.0;
            if (K == NULL) {
                double iso = scatter_source(nq, w, NULL, psi_i, 0);
                for (int32_t q = 0; q < nq; ++q) S[q] = iso;
            } else {
                for (int32_t q = 0; q < nq; ++q) S[q] = scatter_source(nq, w, K, psi_i, q);
            }
            for (int32_t q = 0; q < nq; ++q) {
                double u_i = psi_i[q] / rho_i;
                double flux = 0.0;
                for (int32_t f = 0; f < mf; ++f) {
                    int32_t j = face_nbr[(size_t)i * mf + f];
                    if (j == ORACLE_UNUSED_FACE) continue;
                    const double* n = face_normal + ((size_t)i * mf + f) * 2;
                    const double* m = face_mid + ((size_t)i * mf + f) * 2;
                    double s = omega[(size_t)q * 3 + 0] * n[0] + omega[(size_t)q * 3 + 1] * n[1];
                    /* own side: u_i + Psi_i grad u_i . r_ij */
                    double ui_rec = u_i + gx[(size_t)i * nq + q] * (m[0] - centroid[(size_t)i * 2])
                                        + gy[(size_t)i * nq + q] * (m[1] - centroid[(size_t)i * 2 + 1]);
                    double uj_rec;
                    if (j >= 0) {
                        /* far side: u_j + Psi_j grad u_j . r_ji, r_ji from x_j to the same face */
                        int32_t fb = back_slot(j, i, mf, face_nbr);
                        if (fb < 0) {
#pragma omp atomic write
                            failed = 3;
                            uj_rec = 0.0;
                        } else {
                            const double* mj = face_mid + ((size_t)j * mf + fb) * 2;
                            double u_j = psi[(size_t)j * nq + q] / (rho ? rho[j] : 1.0);
                            uj_rec = u_j + gx[(size_t)j * nq + q] * (mj[0] - centroid[(size_t)j * 2])
                                         + gy[(size_t)j * nq + q] * (mj[1] - centroid[(size_t)j * 2 + 1]);
                        }
                    } else {
                        uj_rec = far_u(i, mf, face_nbr, f, nq, q, rho, inflow, inflow_scale,
                                       neumann, psi);
                    }
                    double H = s > 0.0 ? 1.0 : 0.0;
                    flux += s * ui_rec * H + s * uj_rec * (1.0 - H);
                }
                double R = -alpha_t * sigma_t[i] * psi_i[q] + alpha_s * sigma_s[i] * S[q]
                           + (source ? source[i] : 0.0);
                out[(size_t)i * nq + q] = psi_i[q] - dt / area[i] * flux + dt * R;
            }
        }
        free(S);
    }
    return failed ? -1 - failed : 0;
}

/* One Heun step of the second-order scheme: psi_out = (psi_in + L(L(psi_in))) / 2. */
int oracle_step2(int64_t nc, int32_t mf, const int32_t* face_nbr, const double* face_normal,
                 const double* face_mid, const double* centroid, const double* area, int32_t nq,
                 const double* omega, const double* w, const double* K, const double* sigma_t,
                 const double* sigma_s, const double* rho, const double* source,
                 const double* inflow, double inflow_scale, int32_t neumann, double dt,
                 double alpha_t, double alpha_s, int32_t limiter, double vk_k,
                 const double* psi_in, double* psi_out)
{
    if (limiter != 0 && limiter != 1) return -1;
    if (nc < 0 || mf < 1 || nq < 1 || !face_nbr || !face_normal || !face_mid || !centroid ||
        !area || !omega || !w || !sigma_t || !sigma_s || !psi_in || !psi_out)
        return -1;
    size_t n = (size_t)nc * nq;
    double* star = (double*)malloc(sizeof(double) * (n ? n : 1));
    double* gx = (double*)malloc(sizeof(double) * (n ? n : 1));
    double* gy = (double*)malloc(sizeof(double) * (n ? n : 1));
    int rc = (star && gx && gy) ? 0 : -2;
    if (rc == 0)
        rc = stage2(nc, mf, face_nbr, face_normal, face_mid, centroid, area, nq, omega, w, K,
                    sigma_t, sigma_s, rho, source, inflow, inflow_scale, neumann, dt, alpha_t,
                    alpha_s, limiter, vk_k, psi_in, star, gx, gy);
    if (rc == 0)
        rc = stage2(nc, mf, face_nbr, face_normal, face_mid, centroid, area, nq, omega, w, K,
                    sigma_t, sigma_s, rho, source, inflow, inflow_scale, neumann, dt, alpha_t,
                    alpha_s, limiter, vk_k, star, psi_out, gx, gy);
    if (rc == 0)
        for (size_t k = 0; k < n; ++k) psi_out[k] = 0.5 * (psi_in[k] + psi_out[k]);
    free(star);
    free(gx);
    free(gy);
    return rc;
}
