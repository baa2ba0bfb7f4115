// Host set-up of the implicit collision solve for a dense scattering kernel (IMEX step of
// Sec. 4.2 with the scattering operator of eq. SNEqns): one eigendecomposition of the
// kernel-times-weights matrix A = K W, A[q][p] = K[q][p] w_p, shared by every cell.
//
// Each cell solves (a_i I - b_i A) psi' = r_i with its own a_i = 1 + dt alpha_t sigma_t,i and
// b_i = dt alpha_s sigma_s,i.  With A = V diag(lam) V^-1,
//     (a I - b A)^-1 = (1/a) [I + V diag(b lam / (a - b lam)) V^-1],
// two products with fixed nq x nq operands and a per-cell diagonal in between.
//
// A is brought to symmetric form by a diagonal similarity.  If diag(r) A is symmetric for a
// positive r (true for A = K_s D W with K_s symmetric and D a positive diagonal, e.g. a
// symmetric kernel whose columns were normalised), then S = R^{1/2} A R^{-1/2} is symmetric,
// S = Q diag(lam) Q^T with Q orthogonal, and V = R^{-1/2} Q, V^-1 = Q^T R^{1/2}: both have
// condition number sqrt(max r / min r), and lam is real.  Kernels without such an r are
// refused.
//
// The symmetric eigenproblem is solved in FP64 by Householder reduction to tridiagonal form
// followed by implicitly shifted QR sweeps with Wilkinson's shift (bulge chasing with Givens
// rotations), the textbook dense symmetric eigensolver.
#include <algorithm>
#include <cmath>
#include <limits>
#include <random>
#include <string>
#include <vector>

#include "snrt_internal.h"

namespace snrt {
namespace {

// Householder reduction T = Qt A Qt^T of the symmetric n x n matrix A (row-major, destroyed):
// d = diag(T), e[k] = T[k+1][k]; qt (row-major) receives Q^T = H_{n-3} ... H_0.
void householder_tridiagonal(int n, std::vector<double>& A, std::vector<double>& d,
                             std::vector<double>& e, std::vector<double>& qt) {
    d.assign(n, 0.0);
    e.assign(n > 0 ? n - 1 : 0, 0.0);
    qt.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) qt[(size_t)i * n + i] = 1.0;
    std::vector<double> v(n), p(n), t(n);
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;                       // length of the column below the diagonal
        double* col = v.data();
        double tail = 0.0;
        for (int i = 0; i < m; ++i) {
            col[i] = A[(size_t)(k + 1 + i) * n + k];
            if (i > 0) tail += col[i] * col[i];
        }
        if (tail == 0.0) {                             // already tridiagonal in this column
            e[k] = col[0];
            continue;
        }
        const double norm = std::sqrt(col[0] * col[0] + tail);
        const double alpha = -std::copysign(norm, col[0]);
        col[0] -= alpha;                               // v = x - alpha e1, no cancellation
        const double vn = std::sqrt(col[0] * col[0] + tail);
        for (int i = 0; i < m; ++i) col[i] /= vn;
        e[k] = alpha;
        // trailing block B = A[k+1.., k+1..]:  B <- H B H = B - 2 (v w^T + w v^T),
        // p = B v, w = p - (v.p) v
        double vp = 0.0;
        for (int i = 0; i < m; ++i) {
            const double* row = &A[(size_t)(k + 1 + i) * n + k + 1];
            double s = 0.0;
            for (int j = 0; j < m; ++j) s += row[j] * col[j];
            p[i] = s;
            vp += col[i] * s;
        }
        for (int i = 0; i < m; ++i) p[i] -= vp * col[i];
        for (int i = 0; i < m; ++i) {
            double* row = &A[(size_t)(k + 1 + i) * n + k + 1];
            const double vi = 2.0 * col[i], wi = 2.0 * p[i];
            for (int j = 0; j < m; ++j) row[j] -= vi * p[j] + wi * col[j];
        }
        // Qt <- H Qt on rows k+1..n-1:  t = v^T Qt_rows, Qt_rows -= 2 v t^T
        std::fill(t.begin(), t.end(), 0.0);
        for (int i = 0; i < m; ++i) {
            const double* row = &qt[(size_t)(k + 1 + i) * n];
            const double vi = col[i];
            for (int j = 0; j < n; ++j) t[j] += vi * row[j];
        }
        for (int i = 0; i < m; ++i) {
            double* row = &qt[(size_t)(k + 1 + i) * n];
            const double vi = 2.0 * col[i];
            for (int j = 0; j < n; ++j) row[j] -= vi * t[j];
        }
    }
    for (int i = 0; i < n; ++i) d[i] = A[(size_t)i * n + i];
    if (n >= 2) e[n - 2] = A[(size_t)(n - 1) * n + n - 2];
}

// Eigenvalues of the symmetric tridiagonal (d, e) by implicitly shifted QR sweeps; every
// rotation G of the (k, k+1) plane (T <- G^T T G) is applied to rows k, k+1 of zt, so that
// zt = Qt on entry ends with row j = the eigenvector of d[j] (of the original matrix).
bool tridiagonal_qr(int n, std::vector<double>& d, std::vector<double>& e,
                    std::vector<double>& zt) {
    if (n <= 1) return true;
    const double eps = std::numeric_limits<double>::epsilon();
    double anorm = 0.0;
    for (int i = 0; i < n; ++i)
        anorm = std::max(anorm, std::fabs(d[i]) + (i > 0 ? std::fabs(e[i - 1]) : 0.0) +
                                    (i + 1 < n ? std::fabs(e[i]) : 0.0));
    const double floor = eps * anorm;
    auto negligible = [&](int k) {
        return std::fabs(e[k]) <= eps * (std::fabs(d[k]) + std::fabs(d[k + 1])) ||
               std::fabs(e[k]) <= floor;
    };
    int hi = n - 1;
    long sweeps = 0;
    while (hi > 0) {
        if (negligible(hi - 1)) {
            e[hi - 1] = 0.0;
            --hi;
            continue;
        }
        int lo = hi - 1;
        while (lo > 0 && !negligible(lo - 1)) --lo;
        if (lo > 0) e[lo - 1] = 0.0;
        if (++sweeps > 60L * n) return false;
        // Wilkinson's shift: the eigenvalue of the block's trailing 2 x 2 nearer d[hi]
        const double delta = 0.5 * (d[hi - 1] - d[hi]);
        const double eh = e[hi - 1];
        const double den = delta + std::copysign(std::hypot(delta, eh), delta);
        const double mu = d[hi] - eh * eh / den;
        double x = d[lo] - mu, z = e[lo];
        for (int k = lo; k < hi; ++k) {
            // G^T [x, z]^T = [r, 0]^T with G = [[c, s], [-s, c]]
            const double r = std::hypot(x, z);
            double c = 1.0, s = 0.0;
            if (r != 0.0) {
                c = x / r;
                s = -z / r;
            }
            if (k > lo) e[k - 1] = r;                  // the bulge left behind is gone
            const double a = d[k], b = e[k], g = d[k + 1];
            const double cc = c * c, ss = s * s, cs = c * s;
            d[k] = cc * a - 2.0 * cs * b + ss * g;
            d[k + 1] = ss * a + 2.0 * cs * b + cc * g;
            e[k] = cs * (a - g) + (cc - ss) * b;
            if (k + 1 < hi) {                          // new bulge at (k+2, k)
                x = e[k];
                z = -s * e[k + 1];
                e[k + 1] *= c;
            }
            double* z0 = &zt[(size_t)k * n];
            double* z1 = z0 + n;
            for (int j = 0; j < n; ++j) {
                const double u = z0[j], w = z1[j];
                z0[j] = c * u - s * w;
                z1[j] = s * u + c * w;
            }
        }
    }
    return true;
}

}  // namespace

snrt_status implicit_form(int n, const std::vector<double>& A, std::vector<double>& lam,
                          std::vector<double>& x0, std::vector<double>& x1, double* resid,
                          const char* fn) {
    // positive r with diag(r) A symmetric: r_p = r_q A[q][p] / A[p][q] along the nonzero
    // pattern, one root per connected component
    std::vector<double> r(n, 0.0);
    std::vector<int> queue;
    queue.reserve(n);
    for (int root = 0; root < n; ++root) {
        if (r[root] != 0.0) continue;
        r[root] = 1.0;
        queue.assign(1, root);
        for (size_t h = 0; h < queue.size(); ++h) {
            const int q = queue[h];
            for (int p = 0; p < n; ++p) {
                const double aqp = A[(size_t)q * n + p], apq = A[(size_t)p * n + q];
                if (p == q || r[p] != 0.0 || (aqp == 0.0 && apq == 0.0)) continue;
                const double ratio = aqp / apq;
                if (apq == 0.0 || !(ratio > 0.0) || !std::isfinite(ratio)) {
                    set_error(std::string(fn) + ": K W is not similar to a symmetric matrix by a "
                              "positive diagonal (entries " + std::to_string(q) + "," +
                              std::to_string(p) + ")");
                    return SNRT_E_UNSUPPORTED;
                }
                r[p] = r[q] * ratio;
                queue.push_back(p);
            }
        }
    }
    double amax = 0.0;
    for (double a : A) amax = std::max(amax, std::fabs(a));
    std::vector<double> sr(n), S((size_t)n * n);
    for (int i = 0; i < n; ++i) sr[i] = std::sqrt(r[i]);
    for (int q = 0; q < n; ++q)
        for (int p = 0; p < n; ++p) {
            const double u = r[q] * A[(size_t)q * n + p], v = r[p] * A[(size_t)p * n + q];
            if (std::fabs(u - v) > 1e-10 * std::max({std::fabs(u), std::fabs(v), 1e-300})) {
                set_error(std::string(fn) + ": K W is not similar to a symmetric matrix by a "
                          "positive diagonal (entries " + std::to_string(q) + "," +
                          std::to_string(p) + ")");
                return SNRT_E_UNSUPPORTED;
            }
            S[(size_t)q * n + p] = sr[q] * A[(size_t)q * n + p] / sr[p];
        }
    for (int q = 0; q < n; ++q)               // exact symmetry before the reduction
        for (int p = q + 1; p < n; ++p) {
            const double m = 0.5 * (S[(size_t)q * n + p] + S[(size_t)p * n + q]);
            S[(size_t)q * n + p] = S[(size_t)p * n + q] = m;
        }
    std::vector<double> e, zt;
    householder_tridiagonal(n, S, lam, e, zt);
    if (!tridiagonal_qr(n, lam, e, zt)) {
        set_error(std::string(fn) + ": the symmetric QR iteration did not converge");
        return SNRT_E_UNSUPPORTED;
    }
    // V[q][j] = zt[j][q] / sr[q], V^-1[j][q] = zt[j][q] sr[q]; the product operands are
    // x0[q][j] = V^-1[j][q] (moments U = r x0) and x1[j][q] = lam_j V[q][j] (S = U x1)
    x0.assign((size_t)n * n, 0.0);
    x1.assign((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j)
        for (int q = 0; q < n; ++q) {
            const double z = zt[(size_t)j * n + q];
            x0[(size_t)q * n + j] = z * sr[q];
            x1[(size_t)j * n + q] = lam[j] * z / sr[q];
        }
    // residual on two seeded probes: A y against V diag(lam) V^-1 y, relative to |A| |y|
    std::mt19937_64 gen(12345);
    std::uniform_real_distribution<double> uni(-1.0, 1.0);
    double worst = 0.0;
    std::vector<double> y(n), u(n), ay(n), vy(n);
    for (int probe = 0; probe < 2; ++probe) {
        for (double& t : y) t = uni(gen);
        double ynorm = 0.0;
        for (int q = 0; q < n; ++q) {
            double s = 0.0, t = 0.0;
            for (int p = 0; p < n; ++p) s += A[(size_t)q * n + p] * y[p];
            for (int p = 0; p < n; ++p) t += x0[(size_t)p * n + q] * y[p];   // (V^-1 y)_q
            ay[q] = s;
            u[q] = t;
            ynorm += y[q] * y[q];
        }
        double err = 0.0;
        for (int q = 0; q < n; ++q) {
            double s = 0.0;
            for (int j = 0; j < n; ++j) s += u[j] * x1[(size_t)j * n + q];
            err += (s - ay[q]) * (s - ay[q]);
        }
        const double scale = std::max(amax * n, 1e-300) * std::sqrt(ynorm);
        worst = std::max(worst, std::sqrt(err) / scale);
    }
    *resid = worst;
    if (!(worst <= 1e-10)) {
        set_error(std::string(fn) + ": eigendecomposition residual " + std::to_string(worst) +
                  " too large");
        return SNRT_E_UNSUPPORTED;
    }
    return SNRT_OK;
}

}  // namespace snrt

extern "C" snrt_status snrt_kernel_modes(int32_t n, const double* A, double* lam, double* x0,
                                         double* x1, double* resid) {
    snrt::set_error("");
    if (n < 1 || !A || !lam || !x0 || !x1) {
        snrt::set_error("snrt_kernel_modes: NULL array or n < 1");
        return SNRT_E_ARG;
    }
    const size_t n2 = (size_t)n * n;
    for (size_t i = 0; i < n2; ++i)
        if (!std::isfinite(A[i])) {
            snrt::set_error("snrt_kernel_modes: non-finite entry");
            return SNRT_E_ARG;
        }
    std::vector<double> a(A, A + n2), l, v0, v1;
    double r = 0.0;
    const snrt_status s = snrt::implicit_form(n, a, l, v0, v1, &r, "snrt_kernel_modes");
    if (resid) *resid = r;
    if (s != SNRT_OK) return s;
    std::copy(l.begin(), l.end(), lam);
    std::copy(v0.begin(), v0.end(), x0);
    std::copy(v1.begin(), v1.end(), x1);
    return SNRT_OK;
}
