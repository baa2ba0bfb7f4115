// C ABI of the P_N step (Sec. 3.1 P_N closure, Sec. 4.3): set-up of the flux operators on
// the host (FP64) and the per-step entry points.  Declarations in include/snrt.h.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "pn_pattern.h"
#include "snrt_internal.h"

namespace snrt {
namespace {

constexpr double kPi = 3.14159265358979323846;

// Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on the three-term recurrence).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// A_x, A_y = int m m^T Omega_{x,y} with a product rule exact for degree 2N+1 (N+2 Gauss
// nodes in mu, 2N+4 azimuths).
void flux_jacobians(int N, std::vector<double>& ax, std::vector<double>& ay) {
    const int nm = pn::nmom(N);
    std::vector<double> mu, wl;
    gauss_legendre(N + 2, mu, wl);
    const int nphi = 2 * N + 4;
    ax.assign((size_t)nm * nm, 0.0);
    ay.assign((size_t)nm * nm, 0.0);
    std::vector<double> m(nm);
    for (size_t a = 0; a < mu.size(); ++a) {
        const double s = std::sqrt(std::max(0.0, 1.0 - mu[a] * mu[a]));
        for (int b = 0; b < nphi; ++b) {
            const double phi = (b + 0.5) * 2.0 * kPi / nphi;
            const double ox = s * std::sin(phi), oy = s * std::cos(phi);
            const double w = wl[a] * 2.0 * kPi / nphi;
            real_harmonics(N, ox, oy, mu[a], m.data());
            for (int i = 0; i < nm; ++i) {
                const double wx = w * ox * m[i], wy = w * oy * m[i];
                for (int j = 0; j < nm; ++j) {
                    ax[(size_t)i * nm + j] += wx * m[j];
                    ay[(size_t)i * nm + j] += wy * m[j];
                }
            }
        }
    }
}

// Symmetric eigen-decomposition by cyclic Jacobi rotations: A (n x n, row-major) is
// overwritten; returns eigenvalues in lam and eigenvectors as the columns of V.
void jacobi_eigen(int n, std::vector<double>& A, std::vector<double>& V, std::vector<double>& lam) {
    V.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
    double scale = 0.0;
    for (double v : A) scale += v * v;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += a(p, q) * a(p, q);
        if (off <= 1e-32 * scale || off == 0.0) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = a(p, q);
                if (apq == 0.0) continue;
                const double theta = (a(q, q) - a(p, p)) / (2.0 * apq);
                const double t = (theta >= 0.0 ? 1.0 : -1.0) /
                                 (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {          // columns p, q: A J
                    const double akp = a(k, p), akq = a(k, q);
                    a(k, p) = c * akp - s * akq;
                    a(k, q) = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {          // rows p, q: J^T (A J)
                    const double apk = a(p, k), aqk = a(q, k);
                    a(p, k) = c * apk - s * aqk;
                    a(q, k) = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    double& vkp = V[(size_t)k * n + p];
                    double& vkq = V[(size_t)k * n + q];
                    const double x = vkp, y = vkq;
                    vkp = c * x - s * y;
                    vkq = s * x + c * y;
                }
            }
    }
    lam.resize(n);
    for (int i = 0; i < n; ++i) lam[i] = a(i, i);
}

// |A| = V |Lambda| V^T, taken block by block over the classes that A couples (mask selects
// the class bits A preserves: z and y parity for A_x, z and x parity for A_y).
std::vector<double> abs_matrix(int N, const std::vector<double>& A, int mask) {
    const int nm = pn::nmom(N);
    std::vector<double> out((size_t)nm * nm, 0.0);
    for (int key = 0; key < 8; ++key) {
        if ((key & ~mask) != 0) continue;
        std::vector<int> idx;
        for (int j = 0; j < nm; ++j)
            if ((pn::mom(j).cls & mask) == key) idx.push_back(j);
        const int n = (int)idx.size();
        if (n == 0) continue;
        std::vector<double> B((size_t)n * n), V, lam;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                B[(size_t)i * n + j] = 0.5 * (A[(size_t)idx[i] * nm + idx[j]] +
                                              A[(size_t)idx[j] * nm + idx[i]]);
        jacobi_eigen(n, B, V, lam);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int e = 0; e < n; ++e)
                    s += V[(size_t)i * n + e] * std::fabs(lam[e]) * V[(size_t)j * n + e];
                out[(size_t)idx[i] * nm + idx[j]] = s;
            }
    }
    return out;
}

// Largest entry outside the structural pattern (the operators have spectral radius < 1, so
// an absolute bound is a relative one).
double off_pattern(int N, const std::vector<double>& A, bool (*nz)(const pn::Mom&, const pn::Mom&)) {
    const int nm = pn::nmom(N);
    double out = 0.0;
    for (int i = 0; i < nm; ++i)
        for (int j = 0; j < nm; ++j)
            if (!nz(pn::mom(i), pn::mom(j))) out = std::max(out, std::fabs(A[(size_t)i * nm + j]));
    return out;
}

bool nz_ax(const pn::Mom& a, const pn::Mom& b) { return pn::ax_nz(a, b); }
bool nz_ay(const pn::Mom& a, const pn::Mom& b) { return pn::ay_nz(a, b); }
bool nz_abs(const pn::Mom& a, const pn::Mom& b) { return pn::abs_nz(a, b); }

snrt_status build_operators(int N, std::vector<double>& ax, std::vector<double>& ay,
                            std::vector<double>& axa, std::vector<double>& aya) {
    flux_jacobians(N, ax, ay);
    axa = abs_matrix(N, ax, 5);
    aya = abs_matrix(N, ay, 6);
    const double tol = 1e-12;
    if (off_pattern(N, ax, nz_ax) > tol || off_pattern(N, ay, nz_ay) > tol ||
        off_pattern(N, axa, nz_abs) > tol || off_pattern(N, aya, nz_abs) > tol) {
        set_error("snrt_pn: flux operators outside their structural pattern (internal error)");
        return SNRT_E_HIP;
    }
    return SNRT_OK;
}

}  // namespace
}  // namespace snrt

using namespace snrt;

#define SNRT_REQUIRE(cond, code, msg) \
    do {                              \
        if (!(cond)) {                \
            set_error(msg);           \
            return code;              \
        }                             \
    } while (0)

#define SNRT_TRY(expr)                \
    do {                              \
        snrt_status _s = (expr);      \
        if (_s != SNRT_OK) return _s; \
    } while (0)

extern "C" {

snrt_status snrt_pn_operators(int32_t degree, double* ax, double* ay, double* ax_abs,
                              double* ay_abs) {
    set_error("");
    SNRT_REQUIRE(degree >= 0 && degree <= pn::kMaxDegree, SNRT_E_ARG,
                 "snrt_pn_operators: degree out of range");
    std::vector<double> a, b, c, d;
    SNRT_TRY(build_operators(degree, a, b, c, d));
    const size_t n = a.size();
    if (ax) std::copy(a.begin(), a.end(), ax);
    if (ay) std::copy(b.begin(), b.end(), ay);
    if (ax_abs) std::copy(c.begin(), c.end(), ax_abs);
    if (ay_abs) std::copy(d.begin(), d.end(), ay_abs);
    (void)n;
    return SNRT_OK;
}

void snrt_pn_destroy(snrt_pn* p) {
    if (!p) return;
    dev_free(p->w32);
    dev_free(p->w64);
    dev_free(p->sig32);
    dev_free(p->sig64);
    dev_free(p->wsp32);
    dev_free(p->wa16);
    dev_free(p->wae);
    delete p;
}

snrt_status snrt_pn_create(snrt_pn** out, int32_t degree, const double* sigma_l) {
    set_error("");
    SNRT_REQUIRE(out, SNRT_E_ARG, "snrt_pn_create: out is NULL");
    *out = nullptr;
    SNRT_REQUIRE(degree >= 0 && degree <= pn::kMaxDegree, SNRT_E_ARG,
                 "snrt_pn_create: degree out of range");
    const int N = degree, nm = pn::nmom(N);
    std::vector<double> sl(N + 1, 0.0);
    sl[0] = 1.0;
    if (sigma_l) {
        for (int l = 0; l <= N; ++l) {
            SNRT_REQUIRE(is_finite(sigma_l[l]), SNRT_E_NONFINITE,
                         "snrt_pn_create: non-finite sigma_l");
            sl[l] = sigma_l[l];
        }
    }
    snrt_pn* p = new snrt_pn();
    p->degree = N;
    p->nm = nm;
    p->nmp = (nm + 15) / 16 * 16;
    snrt_status s = build_operators(N, p->ax, p->ay, p->ax_abs, p->ay_abs);
    if (s != SNRT_OK) {
        delete p;
        return s;
    }
    p->sig.resize(nm);
    for (int j = 0; j < nm; ++j) p->sig[j] = sl[pn::mom(j).l];

    // coefficient tables, halved: flux_k = sum_m (A_x[k][m] X_m + ... ) / 2; packed for the
    // unrolled kernel, dense for the chunked one
    const std::vector<double>* mats[4] = {&p->ax, &p->ay, &p->ax_abs, &p->ay_abs};
    auto table = [&](bool packed) {
        std::vector<double> tab;
        if (packed) {
            pn::visit_ops(N, [&](int m, int k, int kind) {
                tab.push_back(0.5 * (*mats[kind])[(size_t)k * nm + m]);
            });
        } else {
            tab.assign((size_t)nm * p->nmp * 4, 0.0);
            pn::visit_ops(N, [&](int m, int k, int kind) {
                tab[((size_t)m * p->nmp + k) * 4 + kind] = 0.5 * (*mats[kind])[(size_t)k * nm + m];
            });
        }
        return tab;
    };
    // the matrix-core step's tables (degree 13): sparse A_x / A_y coefficients, then per
    // (z parity, class) the 32 x 64 class block W[i][k] (k < 32: |A_x| on input k of the
    // class, k >= 32: |A_y| on input k - 32; halved, zero past the class), scaled by 2^e_W
    // (largest magnitude into [2^13, 2^14)) and split into FP16 hi + lo, in the lane order of
    // the 32x32x16 products' left operand (lane l: row l % 32, k = 16 s + 8 (l / 32) + [0, 8))
    std::vector<float> wsp;
    std::vector<uint16_t> wa16;
    std::vector<int32_t> wae;
    if (N == pn::kFusedHighDegree) {
        constexpr int NH = pn::kFusedHighDegree;
        using SO = pn::SparseOps<NH>;
        wsp.assign(SO::count, 0.0f);
        int idx = 0;
        pn::visit_ops(N, [&](int m, int k, int kind) {
            const int si = SO::sidx[idx++];
            if (si >= 0) wsp[si] = (float)(0.5 * (*mats[kind])[(size_t)k * nm + m]);
        });
        wa16.assign((size_t)2 * 4 * 4 * 2 * 64 * 8, 0);
        wae.assign(8, 0);
        for (int pz = 0; pz < 2; ++pz)
            for (int lc = 0; lc < 4; ++lc) {
                const int n = pz == 0 ? pn::ClassOrder<NH, 0>::size[lc] : pn::ClassOrder<NH, 1>::size[lc];
                auto at = [&](int t) {
                    return pz == 0 ? pn::ClassOrder<NH, 0>::at(lc, t) : pn::ClassOrder<NH, 1>::at(lc, t);
                };
                std::vector<float> W(32 * 64, 0.0f);
                float wmax = 0.0f;
                for (int i = 0; i < n; ++i)
                    for (int t = 0; t < n; ++t) {
                        const size_t ki = (size_t)at(i) * nm + at(t);
                        W[i * 64 + t] = (float)(0.5 * p->ax_abs[ki]);
                        W[i * 64 + 32 + t] = (float)(0.5 * p->ay_abs[ki]);
                        wmax = std::max({wmax, std::fabs(W[i * 64 + t]), std::fabs(W[i * 64 + 32 + t])});
                    }
                int E = 0;
                (void)std::frexp(wmax, &E);
                const int ew = wmax > 0.0f ? 14 - E : 0;
                wae[pz * 4 + lc] = ew;
                for (int st = 0; st < 4; ++st)
                    for (int lane = 0; lane < 64; ++lane)
                        for (int e = 0; e < 8; ++e) {
                            const int i = lane % 32, k = 16 * st + 8 * (lane / 32) + e;
                            const float x = std::ldexp(W[i * 64 + k], ew);
                            const _Float16 hi = (_Float16)x;
                            const _Float16 lo = (_Float16)(x - (float)hi);
                            const size_t base = ((((size_t)(pz * 4 + lc) * 4 + st) * 2) * 64 + lane) * 8 + e;
                            wa16[base] = __builtin_bit_cast(uint16_t, hi);
                            wa16[base + 64 * 8] = __builtin_bit_cast(uint16_t, lo);
                        }
            }
    }
    const std::vector<double> t32d = table(pn::has_fused_kernel<float>(N));
    const std::vector<double> tab = table(pn::has_fused_kernel<double>(N));
    std::vector<float> tab32(t32d.begin(), t32d.end());
    std::vector<float> sig32(p->sig.begin(), p->sig.end());
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "snrt_pn_create: hipGetDevice");
    }
    if ((s = dev_alloc(&p->w32, tab32.size(), "P_N coefficients")) != SNRT_OK ||
        (s = dev_alloc(&p->w64, tab.size(), "P_N coefficients")) != SNRT_OK ||
        (s = dev_alloc(&p->sig32, (size_t)nm, "P_N scattering")) != SNRT_OK ||
        (s = dev_alloc(&p->sig64, (size_t)nm, "P_N scattering")) != SNRT_OK ||
        (s = upload(p->w32, tab32.data(), tab32.size(), "snrt_pn_create: upload")) != SNRT_OK ||
        (s = upload(p->w64, tab.data(), tab.size(), "snrt_pn_create: upload")) != SNRT_OK ||
        (s = upload(p->sig32, sig32.data(), (size_t)nm, "snrt_pn_create: upload")) != SNRT_OK ||
        (s = upload(p->sig64, p->sig.data(), (size_t)nm, "snrt_pn_create: upload")) != SNRT_OK ||
        (s = dev_alloc(&p->wsp32, wsp.size(), "P_N sparse coefficients")) != SNRT_OK ||
        (s = upload(p->wsp32, wsp.data(), wsp.size(), "snrt_pn_create: upload")) != SNRT_OK ||
        (s = dev_alloc(&p->wa16, wa16.size(), "P_N class blocks")) != SNRT_OK ||
        (s = upload(p->wa16, wa16.data(), wa16.size(), "snrt_pn_create: upload")) != SNRT_OK ||
        (s = dev_alloc(&p->wae, wae.size(), "P_N class exponents")) != SNRT_OK ||
        (s = upload(p->wae, wae.data(), wae.size(), "snrt_pn_create: upload")) != SNRT_OK) {
        snrt_pn_destroy(p);
        return s;
    }
    *out = p;
    return SNRT_OK;
}

snrt_status snrt_pn_info(const snrt_pn* p, int32_t* degree, int32_t* nmoments) {
    set_error("");
    SNRT_REQUIRE(p, SNRT_E_ARG, "snrt_pn_info: NULL handle");
    if (degree) *degree = p->degree;
    if (nmoments) *nmoments = p->nm;
    return SNRT_OK;
}

snrt_status snrt_pn_state_elems(const snrt_mesh* m, const snrt_pn* p, int64_t* elems) {
    set_error("");
    SNRT_REQUIRE(m && p && elems, SNRT_E_ARG, "snrt_pn_state_elems: NULL argument");
    *elems = (m->nc + 63) / 64 * 64 * (int64_t)p->nm;
    return SNRT_OK;
}

snrt_status snrt_pn_layout(const snrt_mesh* m, const snrt_pn* p, int32_t to_user,
                           int32_t elem_bytes, const void* in, void* out, void* stream) {
    set_error("");
    SNRT_REQUIRE(m && p, SNRT_E_ARG, "snrt_pn_layout: NULL handle");
    SNRT_REQUIRE(to_user == 0 || to_user == 1, SNRT_E_ARG, "snrt_pn_layout: direction must be 0 or 1");
    SNRT_REQUIRE(elem_bytes == 4 || elem_bytes == 8, SNRT_E_ARG,
                 "snrt_pn_layout: elem_bytes must be 4 or 8");
    SNRT_TRY(check_device(m->device, "snrt_pn_layout"));
    SNRT_REQUIRE(p->device == m->device, SNRT_E_ARG, "snrt_pn_layout: handles on different devices");
    if (m->nc == 0) return SNRT_OK;
    SNRT_REQUIRE(in && out, SNRT_E_ARG, "snrt_pn_layout: NULL array");
    const size_t user = (size_t)m->nc * p->nm * elem_bytes;
    const size_t tiled = (size_t)((m->nc + 63) / 64 * 64) * p->nm * elem_bytes;
    SNRT_REQUIRE(!ranges_overlap(in, to_user ? tiled : user, out, to_user ? user : tiled),
                 SNRT_E_ALIAS, "snrt_pn_layout: out aliases in");
    hipError_t e = launch_pn_layout(*m, p->nm, to_user, elem_bytes, in, out,
                                    static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SNRT_OK : hip_fail(e, "snrt_pn_layout: launch");
}

}  // extern "C"

namespace {

template <typename ArgsT>
snrt_status check_pn_step(const char* fn, const snrt_mesh* m, const snrt_pn* p, const ArgsT* a,
                          size_t elem, const void* in, void* out) {
    SNRT_REQUIRE(m && p && a, SNRT_E_ARG, std::string(fn) + ": NULL handle or args");
    SNRT_TRY(check_device(m->device, fn));
    SNRT_REQUIRE(p->device == m->device, SNRT_E_ARG, std::string(fn) + ": handles on different devices");
    SNRT_REQUIRE(is_finite(a->dt) && is_finite(a->alpha_t) && is_finite(a->alpha_s) &&
                     is_finite(a->inflow_scale),
                 SNRT_E_NONFINITE, std::string(fn) + ": non-finite scalar argument");
    SNRT_REQUIRE(a->boundary == SNRT_BC_DIRICHLET || a->boundary == SNRT_BC_NEUMANN, SNRT_E_ARG,
                 std::string(fn) + ": unknown boundary mode");
    if (m->nc == 0) return SNRT_OK;
    SNRT_REQUIRE(a->sigma_t && a->sigma_s, SNRT_E_ARG, std::string(fn) + ": sigma_t/sigma_s NULL");
    SNRT_REQUIRE(in && out, SNRT_E_ARG, std::string(fn) + ": NULL state pointer");
    SNRT_REQUIRE(aligned16(in) && aligned16(out), SNRT_E_ARG,
                 std::string(fn) + ": state pointers must be 16-byte aligned");
    const size_t bytes = (size_t)((m->nc + 63) / 64 * 64) * p->nm * elem;
    SNRT_REQUIRE(bytes < (size_t(1) << 32), SNRT_E_UNSUPPORTED,
                 std::string(fn) + ": a state array of 4 GiB or more is not supported");
    SNRT_REQUIRE(!ranges_overlap(in, bytes, out, bytes), SNRT_E_ALIAS,
                 std::string(fn) + ": output aliases input");
    SNRT_REQUIRE((size_t)m->nbf * p->nm * elem < (size_t(1) << 31), SNRT_E_UNSUPPORTED,
                 std::string(fn) + ": a ghost-moment array of 2 GiB or more is not supported");
    return SNRT_OK;
}

StepArgs32 pn_args32(const snrt_step_args* a) {
    StepArgs32 r;
    r.sigma_t = a->sigma_t;
    r.sigma_s = a->sigma_s;
    r.inv_rho = a->inv_rho;
    r.source = a->source;
    r.inflow = a->boundary == SNRT_BC_NEUMANN ? nullptr : a->inflow;
    r.inflow_scale = (float)a->inflow_scale;
    r.dt = (float)a->dt;
    r.alpha_t = (float)a->alpha_t;
    r.alpha_s = (float)a->alpha_s;
    r.neumann = a->boundary == SNRT_BC_NEUMANN;
    return r;
}

StepArgs64 pn_args64(const snrt_step_args_f64* a) {
    StepArgs64 r;
    r.sigma_t = a->sigma_t;
    r.sigma_s = a->sigma_s;
    r.inv_rho = a->inv_rho;
    r.source = a->source;
    r.inflow = a->boundary == SNRT_BC_NEUMANN ? nullptr : a->inflow;
    r.inflow_scale = a->inflow_scale;
    r.dt = a->dt;
    r.alpha_t = a->alpha_t;
    r.alpha_s = a->alpha_s;
    r.neumann = a->boundary == SNRT_BC_NEUMANN;
    return r;
}

}  // namespace

extern "C" {

snrt_status snrt_pn_step(const snrt_mesh* m, const snrt_pn* p, const snrt_step_args* a,
                         const float* u_in, float* u_out, void* stream) {
    set_error("");
    SNRT_TRY(check_pn_step("snrt_pn_step", m, p, a, sizeof(float), u_in, u_out));
    if (m->nc == 0) return SNRT_OK;
    hipError_t e = launch_pn32(*m, *p, pn_args32(a), u_in, u_out, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SNRT_OK : hip_fail(e, "snrt_pn_step: launch");
}

snrt_status snrt_pn_step_f64(const snrt_mesh* m, const snrt_pn* p, const snrt_step_args_f64* a,
                             const double* u_in, double* u_out, void* stream) {
    set_error("");
    SNRT_TRY(check_pn_step("snrt_pn_step_f64", m, p, a, sizeof(double), u_in, u_out));
    if (m->nc == 0) return SNRT_OK;
    hipError_t e = launch_pn64(*m, *p, pn_args64(a), u_in, u_out, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SNRT_OK : hip_fail(e, "snrt_pn_step_f64: launch");
}

}  // extern "C"
