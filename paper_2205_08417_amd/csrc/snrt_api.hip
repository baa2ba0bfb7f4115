// C ABI of libsnrt: argument validation, handle lifetime, mesh renumbering and launches.
// Declarations and the meaning of every argument are in include/snrt.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <type_traits>
#include <vector>

#include "snrt_internal.h"

namespace snrt {

namespace {
thread_local std::string g_last_error;

// Hilbert index of (x, y) on a 2^16 x 2^16 grid (the standard quadrant-rotation recursion).
uint64_t hilbert_index(uint32_t x, uint32_t y) {
    const uint32_t n = 1u << 16;
    uint64_t d = 0;
    for (uint32_t s = n >> 1; s > 0; s >>= 1) {
        const uint32_t rx = (x & s) ? 1u : 0u;
        const uint32_t ry = (y & s) ? 1u : 0u;
        d += (uint64_t)s * s * ((3u * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) {
                x = n - 1 - x;
                y = n - 1 - y;
            }
            std::swap(x, y);
        }
    }
    return d;
}

}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

const Tune& tune() {
    static const Tune t = [] {
        Tune r;
        if (const char* e = std::getenv("SNRT_STEP_TUNE")) {
            int bpc = 0, bpc2 = 0, bpc3 = 0;
            const int n = std::sscanf(e, "%d,%d,%d", &bpc, &bpc2, &bpc3);
            if (n >= 1 && bpc >= 1 && bpc <= 64) r.step_blocks_per_cu = bpc;
            if (n >= 2 && bpc2 >= 1 && bpc2 <= 64) r.flux2_blocks_per_cu = bpc2;
            if (n >= 3 && bpc3 >= 1 && bpc3 <= 64) r.adjoint_blocks_per_cu = bpc3;
        }
        if (const char* e = std::getenv("SNRT_GEMM_STAGGER")) r.gemm_stagger = std::atoi(e) != 0;
        if (const char* e = std::getenv("SNRT_GEMM_EPILOGUE")) r.gemm_epilogue = std::atoi(e) != 0;
        if (const char* e = std::getenv("SNRT_PN_MFMA")) r.pn_mfma = std::atoi(e) != 0;
        if (const char* e = std::getenv("SNRT_STEP_FUSED")) r.step_fused = std::atoi(e) != 0;
        return r;
    }();
    return t;
}

snrt_status hip_fail(hipError_t e, const char* what) {
    set_error(std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")");
    return SNRT_E_HIP;
}

// Real spherical harmonics m_l^k of the moment equations up to degree N at a direction given
// in the paper's parametrisation (mu = z, phi = atan2(x, y)); out[l*l + l + k].  Built from
// the normalised complex harmonics with associated Legendre functions (Condon-Shortley
// phase) by the three-term recurrence in l: m_l^0 = Y_l^0, m_l^{+-k} = (-1)^k sqrt(2) times
// the real / imaginary part of Y_l^k.
void real_harmonics(int N, double x, double y, double z, double* out) {
    const int W = N + 1;
    std::vector<double> P((size_t)W * W, 0.0);
    auto p = [&](int l, int k) -> double& { return P[(size_t)l * W + k]; };
    const double mu = z;
    const double s = std::sqrt(std::max(0.0, 1.0 - mu * mu));
    const double phi = std::atan2(x, y);
    p(0, 0) = 1.0;
    for (int k = 1; k <= N; ++k) p(k, k) = -(2.0 * k - 1.0) * s * p(k - 1, k - 1);
    for (int k = 0; k < N; ++k) p(k + 1, k) = (2.0 * k + 1.0) * mu * p(k, k);
    for (int k = 0; k <= N; ++k)
        for (int l = k + 2; l <= N; ++l)
            p(l, k) = ((2.0 * l - 1.0) * mu * p(l - 1, k) - (l + k - 1.0) * p(l - 2, k)) / (l - k);
    const double four_pi = 4.0 * 3.14159265358979323846;
    for (int l = 0; l <= N; ++l) {
        double ratio = 1.0;                       // (l-k)!/(l+k)!, built up as k grows
        for (int k = 0; k <= l; ++k) {
            if (k > 0) ratio /= (double)(l + k) * (double)(l - k + 1);
            const double norm = std::sqrt((2.0 * l + 1.0) / four_pi * ratio);
            if (k == 0) {
                out[l * l + l] = norm * p(l, 0);
            } else {
                const double c = ((k & 1) ? -1.0 : 1.0) * std::sqrt(2.0) * norm * p(l, k);
                out[l * l + l + k] = c * std::cos(k * phi);
                out[l * l + l - k] = c * std::sin(k * phi);
            }
        }
    }
}

}  // namespace snrt

using namespace snrt;

#define SNRT_REQUIRE(cond, code, msg) \
    do {                              \
        if (!(cond)) {                \
            set_error(msg);           \
            return code;              \
        }                             \
    } while (0)

#define SNRT_TRY(expr)                       \
    do {                                     \
        snrt_status _s = (expr);             \
        if (_s != SNRT_OK) return _s;        \
    } while (0)

extern "C" {

int snrt_abi_version(void) { return SNRT_ABI_VERSION; }

const char* snrt_last_error(void) { return g_last_error.c_str(); }

// ------------------------------------------------------------------------------------- mesh

void snrt_mesh_destroy(snrt_mesh* m) {
    if (!m) return;
    dev_free(m->geom32);
    dev_free(m->geom64);
    dev_free(m->d_to_user);
    dev_free(m->d_partial);
    dev_free(m->recon32);
    dev_free(m->recon64);
    delete m;
}

snrt_status snrt_mesh_create(snrt_mesh** out, int64_t nc, int32_t mf, const int32_t* face_nbr,
                             const double* face_normal, const double* area,
                             const double* centroid, int64_t nbf, uint32_t flags) {
    g_last_error.clear();
    SNRT_REQUIRE(out, SNRT_E_ARG, "snrt_mesh_create: out is NULL");
    *out = nullptr;
    SNRT_REQUIRE(nc >= 0 && nc < (int64_t)INT32_MAX, SNRT_E_ARG,
                 "snrt_mesh_create: ncells out of range");
    SNRT_REQUIRE(mf == 3 || mf == 4, SNRT_E_UNSUPPORTED, "snrt_mesh_create: max_faces must be 3 or 4");
    SNRT_REQUIRE(nbf >= 0 && nbf < (int64_t)INT32_MAX, SNRT_E_ARG,
                 "snrt_mesh_create: nbfaces out of range");
    SNRT_REQUIRE(flags == SNRT_REORDER_HILBERT || flags == SNRT_NO_REORDER, SNRT_E_ARG,
                 "snrt_mesh_create: unknown flags");
    SNRT_REQUIRE(nc == 0 || (face_nbr && face_normal && area), SNRT_E_ARG,
                 "snrt_mesh_create: NULL mesh array");
    const bool reorder = flags == SNRT_REORDER_HILBERT;
    SNRT_REQUIRE(nc == 0 || !reorder || centroid, SNRT_E_ARG,
                 "snrt_mesh_create: centroids are needed for the Hilbert renumbering");

    // connectivity and geometry checks
    for (int64_t i = 0; i < nc; ++i) {
        SNRT_REQUIRE(is_finite(area[i]) && area[i] > 0.0, SNRT_E_ARG,
                     "snrt_mesh_create: non-positive or non-finite area at cell " + std::to_string(i));
        int used = 0;
        for (int f = 0; f < mf; ++f) {
            const int32_t j = face_nbr[i * mf + f];
            if (j == kUnusedFace) continue;
            ++used;
            const double nx = face_normal[(i * mf + f) * 2], ny = face_normal[(i * mf + f) * 2 + 1];
            SNRT_REQUIRE(is_finite(nx) && is_finite(ny), SNRT_E_ARG,
                         "snrt_mesh_create: non-finite face normal at cell " + std::to_string(i));
            if (j >= 0) {
                SNRT_REQUIRE(j < nc && j != i, SNRT_E_ARG,
                             "snrt_mesh_create: bad neighbour index at cell " + std::to_string(i));
                bool back = false;
                for (int g = 0; g < mf; ++g) back |= face_nbr[(int64_t)j * mf + g] == (int32_t)i;
                SNRT_REQUIRE(back, SNRT_E_ARG,
                             "snrt_mesh_create: adjacency not symmetric at cell " + std::to_string(i));
            } else {
                const int64_t b = -1 - (int64_t)j;
                SNRT_REQUIRE(b < nbf, SNRT_E_ARG,
                             "snrt_mesh_create: boundary face id >= nbfaces at cell " + std::to_string(i));
            }
        }
        SNRT_REQUIRE(used >= 1, SNRT_E_ARG, "snrt_mesh_create: cell without faces");
    }

    // internal order: Hilbert curve through the centroids' bounding box
    std::vector<int64_t> to_user(nc);
    std::iota(to_user.begin(), to_user.end(), 0);
    if (reorder && nc > 1) {
        double x0 = centroid[0], x1 = centroid[0], y0 = centroid[1], y1 = centroid[1];
        for (int64_t i = 0; i < nc; ++i) {
            SNRT_REQUIRE(is_finite(centroid[2 * i]) && is_finite(centroid[2 * i + 1]), SNRT_E_ARG,
                         "snrt_mesh_create: non-finite centroid");
            x0 = std::min(x0, centroid[2 * i]);
            x1 = std::max(x1, centroid[2 * i]);
            y0 = std::min(y0, centroid[2 * i + 1]);
            y1 = std::max(y1, centroid[2 * i + 1]);
        }
        const double span = std::max(std::max(x1 - x0, y1 - y0), 1e-300);
        std::vector<uint64_t> key(nc);
        for (int64_t i = 0; i < nc; ++i) {
            const double fx = (centroid[2 * i] - x0) / span, fy = (centroid[2 * i + 1] - y0) / span;
            const uint32_t ix = (uint32_t)std::min(65535.0, std::floor(fx * 65536.0));
            const uint32_t iy = (uint32_t)std::min(65535.0, std::floor(fy * 65536.0));
            key[i] = hilbert_index(ix, iy);
        }
        std::stable_sort(to_user.begin(), to_user.end(),
                         [&](int64_t a, int64_t b) { return key[a] < key[b]; });
    }
    std::vector<int64_t> to_int(nc);
    for (int64_t k = 0; k < nc; ++k) to_int[to_user[k]] = k;

    std::vector<CellGeom32> g32(nc);
    std::vector<CellGeom64> g64(nc);
    for (int64_t k = 0; k < nc; ++k) {
        const int64_t i = to_user[k];
        CellGeom32& a = g32[k];
        CellGeom64& b = g64[k];
        std::memset(&a, 0, sizeof(a));
        std::memset(&b, 0, sizeof(b));
        for (int f = 0; f < 4; ++f) {
            int32_t j = f < mf ? face_nbr[i * mf + f] : kUnusedFace;
            if (j >= 0) j = (int32_t)to_int[j];
            // an unused slot becomes a face to the cell itself with a zero normal: it then
            // contributes nothing to the flux and needs no special case in the kernels
            if (j == kUnusedFace) j = (int32_t)k;
            a.nbr[f] = b.nbr[f] = j;
            if (f < mf && face_nbr[i * mf + f] != kUnusedFace) {
                b.n[f][0] = face_normal[(i * mf + f) * 2];
                b.n[f][1] = face_normal[(i * mf + f) * 2 + 1];
                a.n[f][0] = (float)b.n[f][0];
                a.n[f][1] = (float)b.n[f][1];
            }
        }
        b.area = area[i];
        b.inv_area = 1.0 / area[i];
        a.area = (float)area[i];
        a.inv_area = (float)(1.0 / area[i]);
    }

    snrt_mesh* m = new snrt_mesh();
    hipError_t e = hipGetDevice(&m->device);
    if (e != hipSuccess) {
        delete m;
        return hip_fail(e, "snrt_mesh_create: hipGetDevice");
    }
    e = hipDeviceGetAttribute(&m->num_cu, hipDeviceAttributeMultiprocessorCount, m->device);
    if (e != hipSuccess || m->num_cu <= 0) {
        delete m;
        return hip_fail(e, "snrt_mesh_create: compute unit count");
    }
    m->nc = nc;
    m->nbf = nbf;
    m->mf = mf;
    m->to_user = std::move(to_user);
    m->face_nbr_user.assign(face_nbr, face_nbr + nc * mf);
    if (centroid) m->centroid_user.assign(centroid, centroid + nc * 2);
    m->n_partial = std::max<int64_t>((nc + kCellsPerBlock - 1) / kCellsPerBlock, 16);
    snrt_status s = SNRT_OK;
    if ((s = dev_alloc(&m->geom32, nc, "geometry")) != SNRT_OK ||
        (s = dev_alloc(&m->geom64, nc, "geometry")) != SNRT_OK ||
        (s = dev_alloc(&m->d_to_user, nc, "permutation")) != SNRT_OK ||
        (s = dev_alloc(&m->d_partial, std::max<int64_t>(m->n_partial, 1), "partials")) != SNRT_OK ||
        (s = upload(m->geom32, g32.data(), nc, "snrt_mesh_create: upload")) != SNRT_OK ||
        (s = upload(m->geom64, g64.data(), nc, "snrt_mesh_create: upload")) != SNRT_OK ||
        (s = upload(m->d_to_user, m->to_user.data(), nc, "snrt_mesh_create: upload")) != SNRT_OK) {
        snrt_mesh_destroy(m);
        return s;
    }
    *out = m;
    return SNRT_OK;
}

snrt_status snrt_mesh_set_face_midpoints(snrt_mesh* m, const double* face_mid) {
    g_last_error.clear();
    SNRT_REQUIRE(m, SNRT_E_ARG, "snrt_mesh_set_face_midpoints: NULL mesh");
    const int64_t nc = m->nc;
    const int32_t mf = m->mf;
    SNRT_REQUIRE(nc == 0 || face_mid, SNRT_E_ARG, "snrt_mesh_set_face_midpoints: NULL face_mid");
    SNRT_REQUIRE(nc == 0 || (int64_t)m->centroid_user.size() == 2 * nc, SNRT_E_ARG,
                 "snrt_mesh_set_face_midpoints: the mesh was created without centroids");
    SNRT_TRY(check_device(m->device, "snrt_mesh_set_face_midpoints"));
    const std::vector<int32_t>& nbr = m->face_nbr_user;
    const std::vector<double>& cen = m->centroid_user;
    std::vector<CellRecon32> r32(nc);
    std::vector<CellRecon64> r64(nc);
    for (int64_t k = 0; k < nc; ++k) {
        const int64_t i = m->to_user[k];
        CellRecon64& b = r64[k];
        CellRecon32& a = r32[k];
        std::memset(&a, 0, sizeof(a));
        std::memset(&b, 0, sizeof(b));
        for (int f = 0; f < mf; ++f) {
            const int32_t j = nbr[i * mf + f];
            if (j == kUnusedFace) continue;
            const double* mid = face_mid + (i * mf + f) * 2;
            SNRT_REQUIRE(is_finite(mid[0]) && is_finite(mid[1]), SNRT_E_ARG,
                         "snrt_mesh_set_face_midpoints: non-finite midpoint at cell " +
                             std::to_string(i));
            b.r_own[f][0] = mid[0] - cen[2 * i];
            b.r_own[f][1] = mid[1] - cen[2 * i + 1];
            if (j >= 0) {
                int g = 0;
                while (g < mf && nbr[(int64_t)j * mf + g] != (int32_t)i) ++g;
                // adjacency was checked symmetric at creation, so the back slot exists
                const double* mj = face_mid + ((int64_t)j * mf + g) * 2;
                SNRT_REQUIRE(is_finite(mj[0]) && is_finite(mj[1]), SNRT_E_ARG,
                             "snrt_mesh_set_face_midpoints: non-finite midpoint at cell " +
                                 std::to_string(j));
                b.r_far[f][0] = mj[0] - cen[2 * (int64_t)j];
                b.r_far[f][1] = mj[1] - cen[2 * (int64_t)j + 1];
            }
            for (int d = 0; d < 2; ++d) {
                a.r_own[f][d] = (float)b.r_own[f][d];
                a.r_far[f][d] = (float)b.r_far[f][d];
            }
        }
    }
    if (!m->recon32) {
        snrt_status s = SNRT_OK;
        if ((s = dev_alloc(&m->recon32, std::max<int64_t>(nc, 1), "reconstruction vectors")) != SNRT_OK)
            return s;
        if ((s = dev_alloc(&m->recon64, std::max<int64_t>(nc, 1), "reconstruction vectors")) != SNRT_OK) {
            dev_free(m->recon32);
            m->recon32 = nullptr;
            return s;
        }
    }
    snrt_status s = SNRT_OK;
    if ((s = upload(m->recon32, r32.data(), nc, "snrt_mesh_set_face_midpoints: upload")) != SNRT_OK ||
        (s = upload(m->recon64, r64.data(), nc, "snrt_mesh_set_face_midpoints: upload")) != SNRT_OK)
        return s;
    return SNRT_OK;
}

snrt_status snrt_mesh_permutation(const snrt_mesh* m, int64_t* internal_to_user) {
    g_last_error.clear();
    SNRT_REQUIRE(m && (internal_to_user || m->nc == 0), SNRT_E_ARG,
                 "snrt_mesh_permutation: NULL argument");
    if (m->nc) std::memcpy(internal_to_user, m->to_user.data(), sizeof(int64_t) * m->nc);
    return SNRT_OK;
}

snrt_status snrt_mesh_info(const snrt_mesh* m, int64_t* nc, int64_t* nbf, int32_t* mf) {
    g_last_error.clear();
    SNRT_REQUIRE(m, SNRT_E_ARG, "snrt_mesh_info: NULL mesh");
    if (nc) *nc = m->nc;
    if (nbf) *nbf = m->nbf;
    if (mf) *mf = m->mf;
    return SNRT_OK;
}

// ------------------------------------------------------------------------------- quadrature

void snrt_quad_destroy(snrt_quad* q) {
    if (!q) return;
    dev_free(q->tab32);
    dev_free(q->tab64);
    delete q;
}

snrt_status snrt_quad_create(snrt_quad** out, int32_t nq, const double* omega, const double* w) {
    g_last_error.clear();
    SNRT_REQUIRE(out, SNRT_E_ARG, "snrt_quad_create: out is NULL");
    *out = nullptr;
    SNRT_REQUIRE(nq >= 1 && nq <= SNRT_MAX_NQ, SNRT_E_UNSUPPORTED,
                 "snrt_quad_create: nq must be in [1, 1024]");
    SNRT_REQUIRE(omega && w, SNRT_E_ARG, "snrt_quad_create: NULL array");
    const double four_pi = 4.0 * 3.14159265358979323846264338327950288;
    std::vector<double> t64(4 * (size_t)nq);
    for (int32_t q = 0; q < nq; ++q) {
        const double ox = omega[3 * q], oy = omega[3 * q + 1], oz = omega[3 * q + 2];
        SNRT_REQUIRE(is_finite(ox) && is_finite(oy) && is_finite(oz) && is_finite(w[q]) && w[q] > 0.0,
                     SNRT_E_ARG, "snrt_quad_create: non-finite ordinate or non-positive weight");
        t64[q] = ox;
        t64[nq + q] = oy;
        t64[2 * nq + q] = w[q];
        t64[3 * nq + q] = w[q] / four_pi;
    }
    std::vector<float> t32(t64.size());
    for (size_t i = 0; i < t64.size(); ++i) t32[i] = (float)t64[i];
    snrt_quad* qd = new snrt_quad();
    hipError_t e = hipGetDevice(&qd->device);
    if (e != hipSuccess) {
        delete qd;
        return hip_fail(e, "snrt_quad_create: hipGetDevice");
    }
    qd->nq = nq;
    qd->w_host.assign(w, w + nq);
    qd->omega_host.assign(omega, omega + (size_t)nq * 3);
    snrt_status s = SNRT_OK;
    if ((s = dev_alloc(&qd->tab32, t32.size(), "ordinates")) != SNRT_OK ||
        (s = dev_alloc(&qd->tab64, t64.size(), "ordinates")) != SNRT_OK ||
        (s = upload(qd->tab32, t32.data(), t32.size(), "snrt_quad_create: upload")) != SNRT_OK ||
        (s = upload(qd->tab64, t64.data(), t64.size(), "snrt_quad_create: upload")) != SNRT_OK) {
        snrt_quad_destroy(qd);
        return s;
    }
    *out = qd;
    return SNRT_OK;
}

// ------------------------------------------------------------------------------- scattering

void snrt_scatter_destroy(snrt_scatter* sc) {
    if (!sc) return;
    for (GemmOperand* ops : {sc->B.fwd, sc->B.adj, sc->B.imp})
        for (int i = 0; i < 2; ++i) {
            dev_free(ops[i].f32);
            dev_free(ops[i].f64);
            dev_free(ops[i].hi);
            dev_free(ops[i].lo);
            dev_free(ops[i].t32);
        }
    dev_free(sc->B.msig32);
    dev_free(sc->B.msig64);
    dev_free(sc->B.lam32);
    dev_free(sc->B.lam64);
    delete sc;
}

snrt_status snrt_scatter_isotropic(snrt_scatter** out, const snrt_quad* q) {
    g_last_error.clear();
    SNRT_REQUIRE(out && q, SNRT_E_ARG, "snrt_scatter_isotropic: NULL argument");
    snrt_scatter* sc = new snrt_scatter();
    sc->device = q->device;
    sc->dense = false;
    sc->B.nq = q->nq;
    *out = sc;
    return SNRT_OK;
}

}  // extern "C"

namespace {

bool low_precision(snrt_precision p) {
    return p == SNRT_BF16X3 || p == SNRT_BF16X2 || p == SNRT_BF16X1 || p == SNRT_FP16X3;
}

bool known_precision(snrt_precision p) { return p == SNRT_FP32 || low_precision(p); }

// Upload X [K][N] (host FP64) in FP64, FP32 and, for the BF16 / FP16 modes, as tiled hi/lo
// parts over N padded with zero columns to a multiple of 128 (FP16: of X * 2^eb, with eb
// putting max |X| into [2^13, 2^14)).
snrt_status make_operand(GemmOperand& op, const std::vector<double>& x, int32_t K, int32_t N,
                         snrt_precision precision, const char* fn) {
    const size_t n = (size_t)K * N;
    op.K = K;
    op.N = N;
    op.Np = ((N + 127) / 128) * 128;
    std::vector<float> x32(n);
    for (size_t i = 0; i < n; ++i) x32[i] = (float)x[i];
    snrt_status s = SNRT_OK;
    if ((s = dev_alloc(&op.f32, n, "scattering operand")) != SNRT_OK ||
        (s = dev_alloc(&op.f64, n, "scattering operand")) != SNRT_OK ||
        (s = upload(op.f32, x32.data(), n, fn)) != SNRT_OK ||
        (s = upload(op.f64, x.data(), n, fn)) != SNRT_OK)
        return s;
    if (precision == SNRT_FP32) {
        // the matrix-core FP32 product where its shape constraints hold
        if (K % 32 != 0 || N % 128 != 0 || K == 0) return SNRT_OK;
        if ((s = dev_alloc(&op.t32, n, "scattering operand (FP32 tiled)")) != SNRT_OK) return s;
        hipError_t e = launch_tile_f32(op.f32, op.t32, K, N, nullptr);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        return e == hipSuccess ? SNRT_OK : hip_fail(e, fn);
    }
    const size_t np = (size_t)K * op.Np;
    std::vector<float> xp(np, 0.0f);
    double mx = 0.0;
    for (int32_t k = 0; k < K; ++k)
        for (int32_t j = 0; j < N; ++j) {
            xp[(size_t)k * op.Np + j] = x32[(size_t)k * N + j];
            mx = std::max(mx, std::fabs(x[(size_t)k * N + j]));
        }
    if (precision == SNRT_FP16X3 && mx > 0.0) {
        int E = 0;
        (void)std::frexp((double)(float)mx, &E);
        op.eb = 14 - E;
    }
    float* staged = nullptr;
    if ((s = dev_alloc(&op.hi, np, "scattering operand (hi)")) != SNRT_OK ||
        (s = dev_alloc(&op.lo, np, "scattering operand (lo)")) != SNRT_OK ||
        (s = dev_alloc(&staged, np, "scattering operand (staging)")) != SNRT_OK)
        return s;
    if ((s = upload(staged, xp.data(), np, fn)) != SNRT_OK) {
        dev_free(staged);
        return s;
    }
    hipError_t e = precision == SNRT_FP16X3
                       ? launch_split_f16(staged, op.hi, op.lo, K, op.Np, op.eb, nullptr)
                       : launch_split_bf16(staged, op.hi, op.lo, K, op.Np, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    dev_free(staged);
    return e == hipSuccess ? SNRT_OK : hip_fail(e, fn);
}

}  // namespace

extern "C" {

snrt_status snrt_scatter_dense(snrt_scatter** out, const snrt_quad* q, const double* K,
                               snrt_precision precision) {
    g_last_error.clear();
    SNRT_REQUIRE(out && q && K, SNRT_E_ARG, "snrt_scatter_dense: NULL argument");
    *out = nullptr;
    SNRT_REQUIRE(known_precision(precision), SNRT_E_ARG, "snrt_scatter_dense: unknown precision");
    const int32_t nq = q->nq;
    if (low_precision(precision)) {
        SNRT_REQUIRE(nq % 32 == 0, SNRT_E_UNSUPPORTED,
                     "snrt_scatter_dense: the BF16 and FP16 modes need nq % 32 == 0");
    }
    SNRT_TRY(check_device(q->device, "snrt_scatter_dense"));
    const size_t n2 = (size_t)nq * nq;
    std::vector<double> b64(n2), bt64(n2);
    for (int32_t p = 0; p < nq; ++p)
        for (int32_t qq = 0; qq < nq; ++qq) {
            const double kqp = K[(size_t)qq * nq + p];
            SNRT_REQUIRE(is_finite(kqp), SNRT_E_ARG, "snrt_scatter_dense: non-finite kernel entry");
            b64[(size_t)p * nq + qq] = q->w_host[p] * kqp;                        // w_p K[q][p]
            bt64[(size_t)p * nq + qq] = q->w_host[qq] * K[(size_t)p * nq + qq];   // w_q K[p][q]
        }
    snrt_scatter* sc = new snrt_scatter();
    sc->device = q->device;
    sc->dense = true;
    DenseB& B = sc->B;
    B.nq = nq;
    B.precision = precision;
    B.chain = 1;
    snrt_status s = SNRT_OK;
    if ((s = make_operand(B.fwd[0], b64, nq, nq, precision, "snrt_scatter_dense: upload")) != SNRT_OK ||
        (s = make_operand(B.adj[0], bt64, nq, nq, precision, "snrt_scatter_dense: upload")) != SNRT_OK) {
        snrt_scatter_destroy(sc);
        return s;
    }
    *out = sc;
    return SNRT_OK;
}

snrt_status snrt_scatter_moments(snrt_scatter** out, const snrt_quad* q, int32_t degree,
                                 const double* sigma_l, snrt_precision precision) {
    g_last_error.clear();
    SNRT_REQUIRE(out && q && sigma_l, SNRT_E_ARG, "snrt_scatter_moments: NULL argument");
    *out = nullptr;
    SNRT_REQUIRE(known_precision(precision), SNRT_E_ARG,
                 "snrt_scatter_moments: unknown precision");
    SNRT_REQUIRE(degree >= 0 && degree <= 30, SNRT_E_ARG,
                 "snrt_scatter_moments: degree must be in [0, 30]");
    const int32_t nq = q->nq;
    if (low_precision(precision)) {
        SNRT_REQUIRE(nq % 32 == 0, SNRT_E_UNSUPPORTED,
                     "snrt_scatter_moments: the BF16 and FP16 modes need nq % 32 == 0");
    }
    for (int l = 0; l <= degree; ++l)
        SNRT_REQUIRE(is_finite(sigma_l[l]), SNRT_E_ARG,
                     "snrt_scatter_moments: non-finite Legendre moment");
    SNRT_TRY(check_device(q->device, "snrt_scatter_moments"));
    const int32_t nm = (degree + 1) * (degree + 1);
    // the low-precision products take their inner width in chunks of 32: the moments are
    // padded with zeros to a multiple of 32 (their outer width is padded to the tile width
    // inside the operand, and only the mid real columns are written)
    const int32_t mid = precision == SNRT_FP32 ? nm : ((nm + 31) / 32) * 32;
    // Mt[q][j] = w_q m_j(Omega_q), Ot[j][q] = sigma_l(j) m_j(Omega_q); zero past nm
    std::vector<double> mt((size_t)nq * mid, 0.0), ot((size_t)mid * nq, 0.0);
    std::vector<double> mtT((size_t)mid * nq, 0.0), otT((size_t)nq * mid, 0.0);
    std::vector<double> m(nm);
    // Gram matrix G = M O of the harmonics under the quadrature (the identity when the rule
    // integrates their products exactly); skipped as too costly above ~2e8 terms
    const bool gram = (double)nm * nm * nq <= 2e8;
    std::vector<double> G(gram ? (size_t)nm * nm : 0, 0.0);
    for (int32_t qq = 0; qq < nq; ++qq) {
        const double* o = q->omega_host.data() + (size_t)qq * 3;
        real_harmonics(degree, o[0], o[1], o[2], m.data());
        if (gram)
            for (int j = 0; j < nm; ++j) {
                const double wj = q->w_host[qq] * m[j];
                for (int k = 0; k < nm; ++k) G[(size_t)j * nm + k] += wj * m[k];
            }
        for (int l = 0; l <= degree; ++l)
            for (int j = l * l; j < (l + 1) * (l + 1); ++j) {
                const double a = q->w_host[qq] * m[j];
                const double b = sigma_l[l] * m[j];
                mt[(size_t)qq * mid + j] = a;
                mtT[(size_t)j * nq + qq] = a;
                ot[(size_t)j * nq + qq] = b;
                otT[(size_t)qq * mid + j] = b;
            }
    }
    snrt_scatter* sc = new snrt_scatter();
    sc->device = q->device;
    sc->dense = true;
    DenseB& B = sc->B;
    B.nq = nq;
    B.precision = precision;
    B.chain = 2;
    B.mid = mid;
    B.degree = degree;
    B.mo_err = gram ? 0.0 : HUGE_VAL;
    for (int j = 0; gram && j < nm; ++j)
        for (int k = 0; k < nm; ++k)
            B.mo_err = std::max(B.mo_err, std::fabs(G[(size_t)j * nm + k] - (j == k ? 1.0 : 0.0)));
    std::vector<double> msig(mid, 0.0);
    std::vector<float> msig32(mid, 0.0f);
    for (int l = 0; l <= degree; ++l)
        for (int j = l * l; j < (l + 1) * (l + 1); ++j) {
            msig[j] = sigma_l[l];
            msig32[j] = (float)sigma_l[l];
        }
    snrt_status s = SNRT_OK;
    const char* fn = "snrt_scatter_moments: upload";
    if ((s = dev_alloc(&B.msig32, (size_t)mid, "moment diagonal")) != SNRT_OK ||
        (s = dev_alloc(&B.msig64, (size_t)mid, "moment diagonal")) != SNRT_OK ||
        (s = upload(B.msig32, msig32.data(), (size_t)mid, fn)) != SNRT_OK ||
        (s = upload(B.msig64, msig.data(), (size_t)mid, fn)) != SNRT_OK ||
        (s = make_operand(B.fwd[0], mt, nq, mid, precision, fn)) != SNRT_OK ||
        (s = make_operand(B.fwd[1], ot, mid, nq, precision, fn)) != SNRT_OK ||
        (s = make_operand(B.adj[0], otT, nq, mid, precision, fn)) != SNRT_OK ||
        (s = make_operand(B.adj[1], mtT, mid, nq, precision, fn)) != SNRT_OK) {
        snrt_scatter_destroy(sc);
        return s;
    }
    *out = sc;
    return SNRT_OK;
}

snrt_status snrt_scatter_prepare_implicit(snrt_scatter* sc) {
    g_last_error.clear();
    const char* fn = "snrt_scatter_prepare_implicit";
    SNRT_REQUIRE(sc, SNRT_E_ARG, std::string(fn) + ": NULL scatter handle");
    SNRT_REQUIRE(sc->dense && sc->B.chain == 1, SNRT_E_UNSUPPORTED,
                 std::string(fn) + ": needs a dense scatter handle (snrt_scatter_dense); "
                 "isotropic and moment-form handles have their own implicit solves");
    DenseB& B = sc->B;
    if (B.implicit) return SNRT_OK;
    SNRT_TRY(check_device(sc->device, fn));
    const int32_t n = B.nq;
    const size_t n2 = (size_t)n * n;
    // the forward operand holds X[p][q] = w_p K[q][p] = A[q][p]
    std::vector<double> X(n2), A(n2);
    hipError_t e = hipMemcpy(X.data(), B.fwd[0].f64, n2 * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, fn);
    for (int32_t p = 0; p < n; ++p)
        for (int32_t q = 0; q < n; ++q) A[(size_t)q * n + p] = X[(size_t)p * n + q];
    std::vector<double> lam, x0, x1;
    double resid = 0.0;
    SNRT_TRY(implicit_form(n, A, lam, x0, x1, &resid, "snrt_scatter_prepare_implicit"));
    std::vector<float> lam32(lam.begin(), lam.end());
    snrt_status s = SNRT_OK;
    if ((s = dev_alloc(&B.lam32, (size_t)n, "implicit eigenvalues")) != SNRT_OK ||
        (s = dev_alloc(&B.lam64, (size_t)n, "implicit eigenvalues")) != SNRT_OK ||
        (s = upload(B.lam32, lam32.data(), (size_t)n, fn)) != SNRT_OK ||
        (s = upload(B.lam64, lam.data(), (size_t)n, fn)) != SNRT_OK ||
        (s = make_operand(B.imp[0], x0, n, n, B.precision, fn)) != SNRT_OK ||
        (s = make_operand(B.imp[1], x1, n, n, B.precision, fn)) != SNRT_OK) {
        for (GemmOperand& op : B.imp) {
            dev_free(op.f32);
            dev_free(op.f64);
            dev_free(op.hi);
            dev_free(op.lo);
            dev_free(op.t32);
            op = GemmOperand();
        }
        dev_free(B.lam32);
        dev_free(B.lam64);
        B.lam32 = nullptr;
        B.lam64 = nullptr;
        return s;
    }
    B.imp_resid = resid;
    B.implicit = true;
    return SNRT_OK;
}

}  // extern "C"

namespace {

// Elements (4 or 8 bytes) of the scattering product's workspace: S [nc][nq], for the moment
// form the moments U [nc][mid] between its two products, and for the FP16 mode the row
// exponents [nc] (int32) of each product's left operand.
size_t product_ws_elems(const snrt_scatter* sc, int64_t nc) {
    if (!sc->dense) return 0;
    return (size_t)nc * (size_t)(sc->B.nq + (sc->B.chain == 2 ? sc->B.mid : 0) +
                                 (sc->B.precision == SNRT_FP16X3 ? 1 : 0));
}

// The IMEX step with a dense kernel's implicit form: the right-hand side's modes U [nc][nq]
// after S [nc][nq], then the FP16 row exponents.
size_t implicit_ws_elems(const snrt_scatter* sc, int64_t nc) {
    if (!sc->dense || !sc->B.implicit) return 0;
    return (size_t)nc * (size_t)(2 * sc->B.nq + (sc->B.precision == SNRT_FP16X3 ? 1 : 0));
}

// snrt_step_dose: the FP32 product workspace, then (16-byte aligned) one FP64 partial sum
// per work item of the step ([nc][items per row]).
size_t dose_ws_offset(const snrt_mesh* m, const snrt_scatter* sc) {
    return (product_ws_elems(sc, m->nc) * sizeof(float) + 15) / 16 * 16;
}
// FP64 dose partials per row: one per work item of the step kernel, or one per 128-ordinate
// piece for the one-launch dense step (whichever is more).
int32_t dose_pieces(const snrt_quad* q, const snrt_scatter* sc) {
    const int32_t items = step_items_per_row(*q, sc->dense);
    return sc->dense && q->nq % 256 == 0 ? std::max(items, q->nq / 128) : items;
}
size_t dose_ws_bytes(const snrt_mesh* m, const snrt_quad* q, const snrt_scatter* sc) {
    return dose_ws_offset(m, sc) + (size_t)m->nc * dose_pieces(q, sc) * sizeof(double);
}

}  // namespace

extern "C" {

snrt_status snrt_workspace_size(const snrt_mesh* m, const snrt_quad* q, const snrt_scatter* sc,
                                size_t* bytes) {
    g_last_error.clear();
    SNRT_REQUIRE(m && q && sc && bytes, SNRT_E_ARG, "snrt_workspace_size: NULL argument");
    SNRT_REQUIRE(sc->B.nq == q->nq, SNRT_E_SHAPE, "snrt_workspace_size: scatter/quad nq differ");
    *bytes = std::max({product_ws_elems(sc, m->nc) * sizeof(double), dose_ws_bytes(m, q, sc),
                       implicit_ws_elems(sc, m->nc) * sizeof(double)});
    return SNRT_OK;
}

snrt_status snrt_step2_workspace_size(const snrt_mesh* m, const snrt_quad* q,
                                      const snrt_scatter* sc, int32_t fp64, size_t* bytes) {
    g_last_error.clear();
    SNRT_REQUIRE(m && q && sc && bytes, SNRT_E_ARG, "snrt_step2_workspace_size: NULL argument");
    SNRT_REQUIRE(fp64 == 0 || fp64 == 1, SNRT_E_ARG, "snrt_step2_workspace_size: fp64 is 0 or 1");
    SNRT_REQUIRE(sc->B.nq == q->nq, SNRT_E_SHAPE,
                 "snrt_step2_workspace_size: scatter/quad nq differ");
    const size_t elem = fp64 ? sizeof(double) : sizeof(float);
    *bytes = ((size_t)m->nc * q->nq * 3 + product_ws_elems(sc, m->nc)) * elem;
    return SNRT_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------------------ steps

namespace {

template <typename ArgsT>
snrt_status check_step_common(const char* fn, const snrt_mesh* m, const snrt_quad* q,
                              const snrt_scatter* sc, const ArgsT* a, size_t elem,
                              const void* in, void* out, void* ws, size_t ws_bytes) {
    SNRT_REQUIRE(m && q && sc && a, SNRT_E_ARG, std::string(fn) + ": NULL handle or args");
    SNRT_REQUIRE(sc->B.nq == q->nq, SNRT_E_SHAPE, std::string(fn) + ": scatter/quad nq differ");
    SNRT_TRY(check_device(m->device, fn));
    SNRT_REQUIRE(q->device == m->device && sc->device == m->device, SNRT_E_ARG,
                 std::string(fn) + ": handles on different devices");
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
    const size_t bytes = (size_t)m->nc * q->nq * elem;
    SNRT_REQUIRE(bytes < (size_t(1) << 32) && (size_t)m->nbf * q->nq * elem < (size_t(1) << 32),
                 SNRT_E_UNSUPPORTED,
                 std::string(fn) + ": a state array of 4 GiB or more is not supported");
    SNRT_REQUIRE(!ranges_overlap(in, bytes, out, bytes), SNRT_E_ALIAS,
                 std::string(fn) + ": output aliases input");
    if (sc->dense) {
        const size_t need = product_ws_elems(sc, m->nc) * elem;
        SNRT_REQUIRE(ws && ws_bytes >= need, SNRT_E_ARG,
                     std::string(fn) + ": dense scattering needs a workspace of " +
                         std::to_string(need) + " bytes");
        SNRT_REQUIRE(aligned16(ws), SNRT_E_ARG, std::string(fn) + ": workspace must be 16-byte aligned");
        SNRT_REQUIRE(!ranges_overlap(ws, need, in, bytes) && !ranges_overlap(ws, need, out, bytes),
                     SNRT_E_ALIAS, std::string(fn) + ": workspace aliases a state array");
    }
    return SNRT_OK;
}

StepArgs32 to32(const snrt_step_args* a) {
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

StepArgs64 to64(const snrt_step_args_f64* a) {
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

// Whether product32 runs this operand on a matrix-core kernel, which applies the epilogue
// modes of GemmEpi (the vector FP32 kernel of odd shapes only stores).
bool product_fuses_epi(const DenseB& B, const GemmOperand& op) {
    if (!tune().gemm_epilogue) return false;
    return B.precision != SNRT_FP32 || op.t32 != nullptr;
}

// out = in X for one right operand of the chain, in the handle's precision; rexp: [M] int32
// scratch for the FP16 mode's row exponents; epi: what happens to each element on the way
// out (product_fuses_epi must hold for any mode but kStore)
hipError_t product32(const DenseB& B, const GemmOperand& op, const float* in, float* out,
                     int64_t M, int32_t* rexp, hipStream_t st, const GemmEpi& epi = GemmEpi()) {
    if (epi.mode != GemmEpi::kStore && !product_fuses_epi(B, op)) return hipErrorNotSupported;
    if (B.precision == SNRT_FP32)
        return op.t32 ? launch_gemm_f32mfma(in, op.t32, out, M, op.K, op.N, st, epi)
                      : launch_gemm32(in, op.f32, out, M, op.K, op.N, st);
    if (B.precision == SNRT_FP16X3)
        return launch_gemm_f16x3(in, op.hi, op.lo, out, M, op.K, op.Np, op.N, rexp, op.eb, st,
                                 epi);
    const int products = B.precision == SNRT_BF16X3 ? 3 : B.precision == SNRT_BF16X2 ? 2 : 1;
    return launch_gemm_bf16(in, op.hi, op.lo, out, M, op.K, op.Np, op.N, products, st, epi);
}

// The FP16 row exponents in the product workspace: after the moments of the moment form.
int32_t* ws_rexp(const DenseB& B, float* after_S, int64_t M) {
    return reinterpret_cast<int32_t*>(after_S + (B.chain == 2 ? (size_t)M * B.mid : 0));
}

// S = Psi B (forward) or G = Lambda B^T (adjoint) into the workspace, FP32 state
// C = A X0 [X1] (forward) or A X0^T-side chain (adjoint); after_S is the workspace past the
// [M][nq] product: the moments between the two products of the moment form ([M][mid]), then
// the FP16 row exponents ([M]).
hipError_t scatter_product32(const snrt_scatter* sc, const float* A, float* C, int64_t M,
                             bool transpose, float* after_S, hipStream_t st) {
    const DenseB& B = sc->B;
    const GemmOperand* ops = transpose ? B.adj : B.fwd;
    int32_t* rexp = after_S ? ws_rexp(B, after_S, M) : nullptr;
    const float* in = A;
    hipError_t e = hipSuccess;
    for (int i = 0; i < B.chain && e == hipSuccess; ++i) {
        float* out = (i == B.chain - 1) ? C : after_S;
        e = product32(B, ops[i], in, out, M, rexp, st);
        in = out;
    }
    return e;
}

// Whether the explicit dense step runs as one launch (the product's last factor with the
// transport update in its epilogue): low-precision products, triangles, nq % 256 == 0.
bool step_fusable(const snrt_mesh& m, const snrt_quad& q, const DenseB& B) {
    if (!tune().step_fused || B.precision == SNRT_FP32 || m.mf != 3 || q.nq % 256 != 0)
        return false;
    const GemmOperand& last = B.fwd[B.chain - 1];
    return last.N == q.nq && last.Np == q.nq && last.K % 32 == 0 && last.hi != nullptr;
}

// The fused dense step: the moment form first writes the moments to after_S (as the
// two-launch step does); the FP16 mode writes the row exponents of the last product's left
// operand, then one launch forms S tile by tile and updates psi_out from it.
hipError_t fused_dense_step(const snrt_mesh& m, const snrt_quad& q, const StepArgs32& a,
                            const DenseB& B, const float* psi_in, float* psi_out,
                            float* after_S, hipStream_t st, double* dpart = nullptr) {
    int32_t* rexp = ws_rexp(B, after_S, m.nc);
    const float* A = psi_in;
    hipError_t e = hipSuccess;
    if (B.chain == 2) {
        e = product32(B, B.fwd[0], psi_in, after_S, m.nc, rexp, st);
        A = after_S;
    }
    const GemmOperand& op = B.fwd[B.chain - 1];
    const int products = B.precision == SNRT_FP16X3 ? 0
                         : B.precision == SNRT_BF16X3 ? 3
                         : B.precision == SNRT_BF16X2 ? 2 : 1;
    if (e == hipSuccess && products == 0) e = launch_row_exp_f16(A, m.nc, op.K, rexp, st);
    if (e != hipSuccess) return e;
    const StepEpi se{m.geom32, q.tab32, a, psi_in, psi_out, m.nc, q.nq, (uint32_t)m.nbf,
                     q.tab64 + 2 * (int64_t)q.nq, dpart};
    return launch_gemm_step(A, op.hi, op.lo, m.nc, op.K, op.Np, products, rexp, op.eb, se, st);
}

// The transposed dense step in one launch, on the same conditions as the forward one for the
// transposed chain's last factor.
bool adjoint_fusable(const snrt_mesh& m, const snrt_quad& q, const DenseB& B) {
    if (!tune().step_fused || B.precision == SNRT_FP32 || m.mf != 3 || q.nq % 256 != 0)
        return false;
    const GemmOperand& last = B.adj[B.chain - 1];
    return last.N == q.nq && last.Np == q.nq && last.K % 32 == 0 && last.hi != nullptr;
}

// The fused transposed step: the moment form's first product into after_G, the FP16 row
// exponents, then one launch forms G tile by tile and updates lam_n from it, leaving the
// gradient sums per 128-ordinate piece in part ([nc][nq / 128][3] floats), which the fold
// adds to the gradients.
template <typename GT>
hipError_t fused_dense_adjoint(const snrt_mesh& m, const snrt_quad& q, const StepArgs32& a,
                               const DenseB& B, const float* psi_n, const float* lam_np1,
                               float* lam_n, GT* g_t, GT* g_s, GT* g_r, float* part,
                               float* after_G, hipStream_t st, const DoseAdj& da) {
    int32_t* rexp = ws_rexp(B, after_G, m.nc);
    const float* A = lam_np1;
    hipError_t e = hipSuccess;
    if (B.chain == 2) {
        e = product32(B, B.adj[0], lam_np1, after_G, m.nc, rexp, st);
        A = after_G;
    }
    const GemmOperand& op = B.adj[B.chain - 1];
    const int products = B.precision == SNRT_FP16X3 ? 0
                         : B.precision == SNRT_BF16X3 ? 3
                         : B.precision == SNRT_BF16X2 ? 2 : 1;
    if (e == hipSuccess && products == 0) e = launch_row_exp_f16(A, m.nc, op.K, rexp, st);
    if (e != hipSuccess) return e;
    const AdjEpi ae{m.geom32, q.tab32, a, psi_n, lam_np1, lam_n, m.nc, q.nq, part, da};
    e = launch_gemm_adjoint(A, op.hi, op.lo, m.nc, op.K, op.Np, products, rexp, op.eb, ae, st);
    if (e != hipSuccess) return e;
    if constexpr (std::is_same<GT, double>::value)
        return launch_adjoint_fold64(m.nc, q.nq / 128, a, part, g_t, g_s, g_r, st);
    else
        return launch_adjoint_fold32(m.nc, q.nq / 128, a, part, g_t, g_s, g_r, st);
}

hipError_t scatter_product64(const snrt_scatter* sc, const double* A, double* C, int64_t M,
                             bool transpose, double* scratch, hipStream_t st) {
    const DenseB& B = sc->B;
    const GemmOperand* ops = transpose ? B.adj : B.fwd;
    const double* in = A;
    hipError_t e = hipSuccess;
    for (int i = 0; i < B.chain && e == hipSuccess; ++i) {
        double* out = (i == B.chain - 1) ? C : scratch;
        e = launch_gemm64(in, ops[i].f64, out, M, ops[i].K, ops[i].N, st);
        in = out;
    }
    return e;
}

}  // namespace

namespace snrt {

snrt_status check_step32(const char* fn, const snrt_mesh* m, const snrt_quad* q,
                         const snrt_scatter* sc, const snrt_step_args* a, const float* in,
                         float* out, void* ws, size_t ws_bytes) {
    return check_step_common(fn, m, q, sc, a, sizeof(float), in, out, ws, ws_bytes);
}

StepArgs32 step_args32(const snrt_step_args* a) { return to32(a); }

// The FP32 adjoint step with gradient accumulators of type GT (float: snrt_step_adjoint;
// double: the reverse pass of long rollouts).
template <typename GT>
snrt_status step_adjoint32_t(const char* fn, const snrt_mesh* m, const snrt_quad* q,
                             const snrt_scatter* sc, const snrt_step_args* a,
                             const float* psi_n, const float* lam_np1, float* lam_n, GT* g_t,
                             GT* g_s, GT* g_r, void* ws, size_t ws_bytes, void* stream,
                             const DoseAdj& da = DoseAdj()) {
    SNRT_TRY(check_step_common(fn, m, q, sc, a, sizeof(float), lam_np1, lam_n, ws, ws_bytes));
    if (m->nc == 0) return SNRT_OK;
    SNRT_REQUIRE(psi_n && aligned16(psi_n), SNRT_E_ARG,
                 std::string(fn) + ": psi_n NULL or misaligned");
    const size_t bytes = (size_t)m->nc * q->nq * sizeof(float);
    SNRT_REQUIRE(!ranges_overlap(psi_n, bytes, lam_n, bytes), SNRT_E_ALIAS,
                 std::string(fn) + ": lam_n aliases psi_n");
    SNRT_REQUIRE(!sc->dense || !ranges_overlap(psi_n, bytes, ws,
                                               product_ws_elems(sc, m->nc) * sizeof(float)),
                 SNRT_E_ALIAS, std::string(fn) + ": workspace aliases psi_n");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const float* G = nullptr;
    if (sc->dense && adjoint_fusable(*m, *q, sc->B)) {
        float* Gbuf = static_cast<float*>(ws);
        const hipError_t e = fused_dense_adjoint(*m, *q, to32(a), sc->B, psi_n, lam_np1, lam_n,
                                                 g_t, g_s, g_r, Gbuf,
                                                 Gbuf + (size_t)m->nc * q->nq, st, da);
        return e == hipSuccess ? SNRT_OK
                               : hip_fail(e, (std::string(fn) + ": fused transposed step").c_str());
    }
    if (sc->dense) {
        float* Gbuf = static_cast<float*>(ws);
        hipError_t e = scatter_product32(sc, lam_np1, Gbuf, m->nc, true,
                                         Gbuf + (size_t)m->nc * q->nq, st);
        if (e != hipSuccess) return hip_fail(e, (std::string(fn) + ": scattering product").c_str());
        G = Gbuf;
    }
    hipError_t e;
    if constexpr (std::is_same<GT, double>::value)
        e = launch_adjoint32_acc64(*m, *q, to32(a), psi_n, lam_np1, lam_n, g_t, g_s, g_r, G, st,
                                   da);
    else
        e = launch_adjoint32(*m, *q, to32(a), psi_n, lam_np1, lam_n, g_t, g_s, g_r, G, st);
    return e == hipSuccess ? SNRT_OK : hip_fail(e, (std::string(fn) + ": launch").c_str());
}

snrt_status step_adjoint32_acc64(const snrt_mesh* m, const snrt_quad* q, const snrt_scatter* sc,
                                 const snrt_step_args* a, const float* psi_n,
                                 const float* lam_np1, float* lam_n, double* g_t, double* g_s,
                                 double* g_r, void* ws, size_t ws_bytes, void* stream,
                                 const DoseAdj& da) {
    return step_adjoint32_t<double>("snrt_rollout_adjoint", m, q, sc, a, psi_n, lam_np1, lam_n,
                                    g_t, g_s, g_r, ws, ws_bytes, stream, da);
}

}  // namespace snrt

extern "C" {

snrt_status snrt_step(const snrt_mesh* m, const snrt_quad* q, const snrt_scatter* sc,
                      const snrt_step_args* a, const float* psi_in, float* psi_out, void* ws,
                      size_t ws_bytes, void* stream) {
    g_last_error.clear();
    SNRT_TRY(check_step_common("snrt_step", m, q, sc, a, sizeof(float), psi_in, psi_out, ws,
                               ws_bytes));
    if (m->nc == 0) return SNRT_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const float* S = nullptr;
    if (sc->dense) {
        float* Sbuf = static_cast<float*>(ws);
        float* after = Sbuf + (size_t)m->nc * q->nq;
        if (step_fusable(*m, *q, sc->B)) {
            const hipError_t e = fused_dense_step(*m, *q, to32(a), sc->B, psi_in, psi_out,
                                                  after, st);
            return e == hipSuccess ? SNRT_OK : hip_fail(e, "snrt_step: fused dense step");
        }
        hipError_t e = scatter_product32(sc, psi_in, Sbuf, m->nc, false, after, st);
        if (e != hipSuccess) return hip_fail(e, "snrt_step: scattering product");
        S = Sbuf;
    }
    hipError_t e = launch_step32(*m, *q, to32(a), psi_in, psi_out, S, st);
    return e == hipSuccess ? SNRT_OK : hip_fail(e, "snrt_step: launch");
}

snrt_status snrt_step_dose(const snrt_mesh* m, const snrt_quad* q, const snrt_scatter* sc,
                           const snrt_step_args* a, const float* psi_in, float* psi_out,
                           double coeff, double* dose, void* ws, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    const char* fn = "snrt_step_dose";
    SNRT_TRY(check_step_common(fn, m, q, sc, a, sizeof(float), psi_in, psi_out, ws, ws_bytes));
    SNRT_REQUIRE(is_finite(coeff), SNRT_E_NONFINITE, "snrt_step_dose: non-finite coeff");
    if (m->nc == 0) return SNRT_OK;
    SNRT_REQUIRE(dose, SNRT_E_ARG, "snrt_step_dose: NULL dose");
    const size_t need = dose_ws_bytes(m, q, sc);
    SNRT_REQUIRE(ws && ws_bytes >= need, SNRT_E_ARG,
                 "snrt_step_dose: needs a workspace of " + std::to_string(need) + " bytes");
    SNRT_REQUIRE(aligned16(ws), SNRT_E_ARG, "snrt_step_dose: workspace must be 16-byte aligned");
    const size_t row = (size_t)m->nc * q->nq * sizeof(float), db = (size_t)m->nc * sizeof(double);
    SNRT_REQUIRE(!ranges_overlap(ws, need, psi_in, row) && !ranges_overlap(ws, need, psi_out, row),
                 SNRT_E_ALIAS, "snrt_step_dose: workspace aliases a state array");
    SNRT_REQUIRE(!ranges_overlap(dose, db, psi_in, row) && !ranges_overlap(dose, db, psi_out, row) &&
                     !ranges_overlap(dose, db, ws, need),
                 SNRT_E_ALIAS, "snrt_step_dose: dose aliases a state array or the workspace");
    hipStream_t st = static_cast<hipStream_t>(stream);
    double* part = reinterpret_cast<double*>(static_cast<char*>(ws) + dose_ws_offset(m, sc));
    const float* S = nullptr;
    if (sc->dense) {
        float* Sbuf = static_cast<float*>(ws);
        float* after = Sbuf + (size_t)m->nc * q->nq;
        if (step_fusable(*m, *q, sc->B)) {
            hipError_t e = fused_dense_step(*m, *q, to32(a), sc->B, psi_in, psi_out, after, st,
                                            part);
            if (e == hipSuccess)
                e = launch_dose_fold(*m, part, q->nq / 128, a->inv_rho, coeff, dose, st);
            return e == hipSuccess ? SNRT_OK : hip_fail(e, "snrt_step_dose: fused dense step");
        }
        hipError_t e = scatter_product32(sc, psi_in, Sbuf, m->nc, false, after, st);
        if (e != hipSuccess) return hip_fail(e, "snrt_step_dose: scattering product");
        S = Sbuf;
    }
    hipError_t e = launch_step32(*m, *q, to32(a), psi_in, psi_out, S, st, part);
    if (e == hipSuccess)
        e = launch_dose_fold(*m, part, step_items_per_row(*q, sc->dense), a->inv_rho, coeff,
                             dose, st);
    return e == hipSuccess ? SNRT_OK : hip_fail(e, "snrt_step_dose: launch");
}

snrt_status snrt_step_f64(const snrt_mesh* m, const snrt_quad* q, const snrt_scatter* sc,
                          const snrt_step_args_f64* a, const double* psi_in, double* psi_out,
                          void* ws, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    SNRT_TRY(check_step_common("snrt_step_f64", m, q, sc, a, sizeof(double), psi_in, psi_out, ws,
                               ws_bytes));
    if (m->nc == 0) return SNRT_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const double* S = nullptr;
    if (sc->dense) {
        double* Sbuf = static_cast<double*>(ws);
        hipError_t e = scatter_product64(sc, psi_in, Sbuf, m->nc, false,
                                         Sbuf + (size_t)m->nc * q->nq, st);
        if (e != hipSuccess) return hip_fail(e, "snrt_step_f64: scattering product");
        S = Sbuf;
    }
    hipError_t e = launch_step64(*m, *q, to64(a), psi_in, psi_out, S, st);
    return e == hipSuccess ? SNRT_OK : hip_fail(e, "snrt_step_f64: launch");
}

snrt_status snrt_step_adjoint(const snrt_mesh* m, const snrt_quad* q, const snrt_scatter* sc,
                              const snrt_step_args* a, const float* psi_n, const float* lam_np1,
                              float* lam_n, float* g_t, float* g_s, float* g_r, void* ws,
                              size_t ws_bytes, void* stream) {
    g_last_error.clear();
    return step_adjoint32_t<float>("snrt_step_adjoint", m, q, sc, a, psi_n, lam_np1, lam_n, g_t,
                                   g_s, g_r, ws, ws_bytes, stream);
}

snrt_status snrt_step_adjoint_f64(const snrt_mesh* m, const snrt_quad* q, const snrt_scatter* sc,
                                  const snrt_step_args_f64* a, const double* psi_n,
                                  const double* lam_np1, double* lam_n, double* g_t, double* g_s,
                                  double* g_r, void* ws, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    SNRT_TRY(check_step_common("snrt_step_adjoint_f64", m, q, sc, a, sizeof(double), lam_np1,
                               lam_n, ws, ws_bytes));
    if (m->nc == 0) return SNRT_OK;
    SNRT_REQUIRE(psi_n && aligned16(psi_n), SNRT_E_ARG,
                 "snrt_step_adjoint_f64: psi_n NULL or misaligned");
    const size_t bytes = (size_t)m->nc * q->nq * sizeof(double);
    SNRT_REQUIRE(!ranges_overlap(psi_n, bytes, lam_n, bytes), SNRT_E_ALIAS,
                 "snrt_step_adjoint_f64: lam_n aliases psi_n");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const double* G = nullptr;
    if (sc->dense) {
        double* Gbuf = static_cast<double*>(ws);
        hipError_t e = scatter_product64(sc, lam_np1, Gbuf, m->nc, true,
                                         Gbuf + (size_t)m->nc * q->nq, st);
        if (e != hipSuccess) return hip_fail(e, "snrt_step_adjoint_f64: scattering product");
        G = Gbuf;
    }
    hipError_t e = launch_adjoint64(*m, *q, to64(a), psi_n, lam_np1, lam_n, g_t, g_s, g_r, G, st);
    return e == hipSuccess ? SNRT_OK : hip_fail(e, "snrt_step_adjoint_f64: launch");
}

}  // extern "C"

namespace {

// Heun step of the second-order scheme on the workspace [star | G (two planes) | S].
template <typename T, typename ArgsT>
snrt_status step2_common(const char* fn, const snrt_mesh* m, const snrt_quad* q,
                         const snrt_scatter* sc, const ArgsT* a, const snrt_limiter* lim_in,
                         const T* psi_in, T* psi_out, void* ws, size_t ws_bytes, void* stream) {
    SNRT_TRY(check_step_common(fn, m, q, sc, a, sizeof(T), psi_in, psi_out, ws, ws_bytes));
    Limiter lim;
    if (lim_in) {
        SNRT_REQUIRE(lim_in->kind == SNRT_LIMITER_BARTH_JESPERSEN ||
                         lim_in->kind == SNRT_LIMITER_VENKATAKRISHNAN,
                     SNRT_E_ARG, std::string(fn) + ": unknown limiter kind");
        SNRT_REQUIRE(lim_in->reserved == 0, SNRT_E_ARG,
                     std::string(fn) + ": limiter.reserved must be 0");
        SNRT_REQUIRE(is_finite(lim_in->k) && lim_in->k >= 0.0, SNRT_E_ARG,
                     std::string(fn) + ": limiter k must be finite and >= 0");
        lim.kind = lim_in->kind;
        lim.k = lim_in->k;
    }
    if (m->nc == 0) return SNRT_OK;
    SNRT_REQUIRE(m->recon32 && m->recon64, SNRT_E_ARG,
                 std::string(fn) + ": call snrt_mesh_set_face_midpoints first");
    const size_t row = (size_t)m->nc * q->nq * sizeof(T);
    const size_t need = row * 3 + product_ws_elems(sc, m->nc) * sizeof(T);
    SNRT_REQUIRE(ws && ws_bytes >= need, SNRT_E_ARG,
                 std::string(fn) + ": needs a workspace of " + std::to_string(need) + " bytes");
    SNRT_REQUIRE(aligned16(ws), SNRT_E_ARG, std::string(fn) + ": workspace must be 16-byte aligned");
    SNRT_REQUIRE(!ranges_overlap(ws, need, psi_in, row) && !ranges_overlap(ws, need, psi_out, row),
                 SNRT_E_ALIAS, std::string(fn) + ": workspace aliases a state array");
    T* star = static_cast<T*>(ws);
    T* G = star + (size_t)m->nc * q->nq;
    T* S = sc->dense ? G + 2 * (size_t)m->nc * q->nq : nullptr;
    T* U = sc->dense ? S + (size_t)m->nc * q->nq : nullptr;     // moments between products
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    const T* in[2] = {psi_in, star};
    T* outp[2] = {star, psi_out};
    for (int stage = 0; stage < 2 && e == hipSuccess; ++stage) {
        if constexpr (sizeof(T) == 4) {
            const StepArgs32 a32 = to32(a);
            e = launch_grad2_32(*m, *q, a32, lim, in[stage], G, st);
            if (e == hipSuccess && S) e = scatter_product32(sc, in[stage], S, m->nc, false, U, st);
            if (e == hipSuccess)
                e = launch_flux2_32(*m, *q, a32, in[stage], G, S, stage ? psi_in : nullptr,
                                    outp[stage], st);
        } else {
            const StepArgs64 a64 = to64(a);
            e = launch_grad2_64(*m, *q, a64, lim, in[stage], G, st);
            if (e == hipSuccess && S) e = scatter_product64(sc, in[stage], S, m->nc, false, U, st);
            if (e == hipSuccess)
                e = launch_flux2_64(*m, *q, a64, in[stage], G, S, stage ? psi_in : nullptr,
                                    outp[stage], st);
        }
    }
    return e == hipSuccess ? SNRT_OK : hip_fail(e, (std::string(fn) + ": launch").c_str());
}

}  // namespace

extern "C" {

snrt_status snrt_step2(const snrt_mesh* m, const snrt_quad* q, const snrt_scatter* sc,
                       const snrt_step_args* a, const float* psi_in, float* psi_out, void* ws,
                       size_t ws_bytes, void* stream) {
    g_last_error.clear();
    return step2_common<float>("snrt_step2", m, q, sc, a, nullptr, psi_in, psi_out, ws,
                               ws_bytes, stream);
}

snrt_status snrt_step2_f64(const snrt_mesh* m, const snrt_quad* q, const snrt_scatter* sc,
                           const snrt_step_args_f64* a, const double* psi_in, double* psi_out,
                           void* ws, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    return step2_common<double>("snrt_step2_f64", m, q, sc, a, nullptr, psi_in, psi_out, ws,
                                ws_bytes, stream);
}

snrt_status snrt_step2_limited(const snrt_mesh* m, const snrt_quad* q, const snrt_scatter* sc,
                               const snrt_step_args* a, const snrt_limiter* lim,
                               const float* psi_in, float* psi_out, void* ws, size_t ws_bytes,
                               void* stream) {
    g_last_error.clear();
    return step2_common<float>("snrt_step2_limited", m, q, sc, a, lim, psi_in, psi_out, ws,
                               ws_bytes, stream);
}

snrt_status snrt_step2_limited_f64(const snrt_mesh* m, const snrt_quad* q,
                                   const snrt_scatter* sc, const snrt_step_args_f64* a,
                                   const snrt_limiter* lim, const double* psi_in,
                                   double* psi_out, void* ws, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    return step2_common<double>("snrt_step2_limited_f64", m, q, sc, a, lim, psi_in, psi_out,
                                ws, ws_bytes, stream);
}

snrt_status snrt_step_imex(const snrt_mesh* m, const snrt_quad* q, const snrt_scatter* sc,
                           const snrt_step_args* a, const float* psi_in, float* psi_out,
                           void* stream) {
    g_last_error.clear();
    SNRT_REQUIRE(sc, SNRT_E_ARG, "snrt_step_imex: NULL scatter handle");
    SNRT_REQUIRE(!sc->dense, SNRT_E_UNSUPPORTED,
                 "snrt_step_imex: only isotropic scattering has the closed-form implicit solve "
                 "(dense kernels: snrt_step_imex_dense; moment form: snrt_step_imex_moments)");
    SNRT_TRY(check_step_common("snrt_step_imex", m, q, sc, a, sizeof(float), psi_in, psi_out,
                               nullptr, 0));
    if (m->nc == 0) return SNRT_OK;
    hipError_t e = launch_imex32(*m, *q, to32(a), psi_in, psi_out, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SNRT_OK : hip_fail(e, "snrt_step_imex: launch");
}

snrt_status snrt_step_imex_f64(const snrt_mesh* m, const snrt_quad* q, const snrt_scatter* sc,
                               const snrt_step_args_f64* a, const double* psi_in,
                               double* psi_out, void* stream) {
    g_last_error.clear();
    SNRT_REQUIRE(sc, SNRT_E_ARG, "snrt_step_imex_f64: NULL scatter handle");
    SNRT_REQUIRE(!sc->dense, SNRT_E_UNSUPPORTED,
                 "snrt_step_imex_f64: only isotropic scattering has the closed-form implicit "
                 "solve (dense kernels: snrt_step_imex_dense_f64; moment form: "
                 "snrt_step_imex_moments_f64)");
    SNRT_TRY(check_step_common("snrt_step_imex_f64", m, q, sc, a, sizeof(double), psi_in,
                               psi_out, nullptr, 0));
    if (m->nc == 0) return SNRT_OK;
    hipError_t e = launch_imex64(*m, *q, to64(a), psi_in, psi_out, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SNRT_OK : hip_fail(e, "snrt_step_imex_f64: launch");
}

}  // extern "C"

namespace {

// Largest |M O - I| for which the moment-form IMEX inverse is taken as exact.
constexpr double kMomentGramTol = 1e-10;

// The IMEX solve in mode space, shared by the moment form and a dense kernel's implicit
// form: r = the collision-free explicit step (into psi_out), U = r X0, U_j *= b / (a - b
// sig_j), S = U X1, psi_out = (r + S) / a.  S [nc][nq] and U [nc][mid] in the workspace,
// rexp [nc] the FP16 row exponents (FP32 state only).
template <typename T, typename ArgsT>
hipError_t imex_modes(const snrt_mesh* m, const snrt_quad* q, const DenseB& B,
                      const GemmOperand* ops, const float* sig32, const double* sig64,
                      int32_t mid, const ArgsT* a, const T* psi_in, T* psi_out, T* S, T* U,
                      int32_t* rexp, hipStream_t st) {
    hipError_t e;
    if constexpr (sizeof(T) == 4) {
        const StepArgs32 a32 = to32(a);
        StepArgs32 free_flight = a32;
        free_flight.alpha_t = 0.0f;
        free_flight.alpha_s = 0.0f;
        e = launch_free_step32(*m, *q, free_flight, psi_in, psi_out, st);
        // the per-cell diagonal and the final combine ride on the two products' epilogues
        // where the matrix-core kernels run them (S then stays unused), else separate passes
        GemmEpi scale;
        scale.mode = GemmEpi::kScale;
        scale.sigma_t = a32.sigma_t;
        scale.sigma_s = a32.sigma_s;
        scale.sig = sig32;
        scale.dt = a32.dt;
        scale.alpha_t = a32.alpha_t;
        scale.alpha_s = a32.alpha_s;
        GemmEpi combine = scale;
        combine.mode = GemmEpi::kCombine;
        combine.sig = nullptr;
        if (e == hipSuccess) {
            if (product_fuses_epi(B, ops[0])) {
                e = product32(B, ops[0], psi_out, U, m->nc, rexp, st, scale);
            } else {
                e = product32(B, ops[0], psi_out, U, m->nc, rexp, st);
                if (e == hipSuccess) e = launch_imex_moment_scale32(a32, U, sig32, m->nc, mid, st);
            }
        }
        if (e == hipSuccess) {
            const GemmOperand& o1 = ops[1];
            if (product_fuses_epi(B, o1) && B.precision != SNRT_FP32 && o1.hi &&
                o1.N == q->nq && o1.Np == q->nq && q->nq % 256 == 0) {
                // the combine on the product's tiles staged in LDS, full rows per wave
                const int products = B.precision == SNRT_FP16X3 ? 0
                                     : B.precision == SNRT_BF16X3 ? 3
                                     : B.precision == SNRT_BF16X2 ? 2 : 1;
                if (products == 0) e = launch_row_exp_f16(U, m->nc, o1.K, rexp, st);
                const CombineEpi ce{a32.sigma_t, a32.dt, a32.alpha_t, psi_out, m->nc, q->nq};
                if (e == hipSuccess)
                    e = launch_gemm_combine(U, o1.hi, o1.lo, m->nc, o1.K, o1.Np, products, rexp,
                                            o1.eb, ce, st);
            } else if (product_fuses_epi(B, o1)) {
                e = product32(B, ops[1], U, psi_out, m->nc, rexp, st, combine);
            } else {
                e = product32(B, ops[1], U, S, m->nc, rexp, st);
                if (e == hipSuccess) e = launch_imex_combine32(a32, psi_out, S, m->nc, q->nq, st);
            }
        }
    } else {
        const StepArgs64 a64 = to64(a);
        StepArgs64 free_flight = a64;
        free_flight.alpha_t = 0.0;
        free_flight.alpha_s = 0.0;
        e = launch_free_step64(*m, *q, free_flight, psi_in, psi_out, st);
        if (e == hipSuccess)
            e = launch_gemm64(psi_out, ops[0].f64, U, m->nc, ops[0].K, ops[0].N, st);
        if (e == hipSuccess) e = launch_imex_moment_scale64(a64, U, sig64, m->nc, mid, st);
        if (e == hipSuccess)
            e = launch_gemm64(U, ops[1].f64, S, m->nc, ops[1].K, ops[1].N, st);
        if (e == hipSuccess) e = launch_imex_combine64(a64, psi_out, S, m->nc, q->nq, st);
    }
    return e;
}

// IMEX with moment-projected scattering: with M O = I the per-cell inverse of a I - b O Sigma M
// is (1/a) [I + O diag(b Sigma / (a - b Sigma)) M].
template <typename T, typename ArgsT>
snrt_status imex_moments_common(const char* fn, const snrt_mesh* m, const snrt_quad* q,
                                const snrt_scatter* sc, const ArgsT* a, const T* psi_in,
                                T* psi_out, void* ws, size_t ws_bytes, void* stream) {
    SNRT_REQUIRE(sc, SNRT_E_ARG, std::string(fn) + ": NULL scatter handle");
    SNRT_REQUIRE(sc->dense && sc->B.chain == 2, SNRT_E_UNSUPPORTED,
                 std::string(fn) + ": needs a moment-form scatter handle (snrt_scatter_moments)");
    SNRT_REQUIRE(sc->B.mo_err <= kMomentGramTol, SNRT_E_UNSUPPORTED,
                 std::string(fn) + ": the quadrature does not integrate the harmonics' products "
                                   "exactly (M O != I), so the closed-form inverse does not hold");
    SNRT_TRY(check_step_common(fn, m, q, sc, a, sizeof(T), psi_in, psi_out, ws, ws_bytes));
    if (m->nc == 0) return SNRT_OK;
    const DenseB& B = sc->B;
    T* S = static_cast<T*>(ws);
    T* U = S + (size_t)m->nc * q->nq;
    int32_t* rexp = nullptr;
    if constexpr (sizeof(T) == 4) rexp = ws_rexp(B, U, m->nc);
    hipError_t e = imex_modes<T>(m, q, B, B.fwd, B.msig32, B.msig64, B.mid, a, psi_in, psi_out,
                                 S, U, rexp, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SNRT_OK : hip_fail(e, (std::string(fn) + ": launch").c_str());
}

// IMEX with a dense kernel (implicit form from snrt_scatter_prepare_implicit): K W =
// V diag(lam) V^-1, so the per-cell inverse is (1/a) [I + V diag(b lam / (a - b lam)) V^-1].
template <typename T, typename ArgsT>
snrt_status imex_dense_common(const char* fn, const snrt_mesh* m, const snrt_quad* q,
                              const snrt_scatter* sc, const ArgsT* a, const T* psi_in,
                              T* psi_out, void* ws, size_t ws_bytes, void* stream) {
    SNRT_REQUIRE(sc, SNRT_E_ARG, std::string(fn) + ": NULL scatter handle");
    SNRT_REQUIRE(sc->dense && sc->B.chain == 1, SNRT_E_UNSUPPORTED,
                 std::string(fn) + ": needs a dense scatter handle (snrt_scatter_dense)");
    SNRT_REQUIRE(sc->B.implicit, SNRT_E_UNSUPPORTED,
                 std::string(fn) + ": the handle has no implicit form "
                                   "(call snrt_scatter_prepare_implicit first)");
    SNRT_TRY(check_step_common(fn, m, q, sc, a, sizeof(T), psi_in, psi_out, ws, ws_bytes));
    if (m->nc == 0) return SNRT_OK;
    const size_t need = implicit_ws_elems(sc, m->nc) * sizeof(T);
    const size_t bytes = (size_t)m->nc * q->nq * sizeof(T);
    SNRT_REQUIRE(ws_bytes >= need, SNRT_E_ARG,
                 std::string(fn) + ": the implicit solve needs a workspace of " +
                     std::to_string(need) + " bytes (snrt_workspace_size after "
                     "snrt_scatter_prepare_implicit)");
    SNRT_REQUIRE(!ranges_overlap(ws, need, psi_in, bytes) && !ranges_overlap(ws, need, psi_out, bytes),
                 SNRT_E_ALIAS, std::string(fn) + ": workspace aliases a state array");
    const DenseB& B = sc->B;
    T* S = static_cast<T*>(ws);
    T* U = S + (size_t)m->nc * q->nq;
    int32_t* rexp = reinterpret_cast<int32_t*>(U + (size_t)m->nc * q->nq);
    hipError_t e = imex_modes<T>(m, q, B, B.imp, B.lam32, B.lam64, B.nq, a, psi_in, psi_out, S,
                                 U, sizeof(T) == 4 ? rexp : nullptr,
                                 static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SNRT_OK : hip_fail(e, (std::string(fn) + ": launch").c_str());
}

}  // namespace

extern "C" {

snrt_status snrt_step_imex_moments(const snrt_mesh* m, const snrt_quad* q,
                                   const snrt_scatter* sc, const snrt_step_args* a,
                                   const float* psi_in, float* psi_out, void* ws,
                                   size_t ws_bytes, void* stream) {
    g_last_error.clear();
    return imex_moments_common<float>("snrt_step_imex_moments", m, q, sc, a, psi_in, psi_out,
                                      ws, ws_bytes, stream);
}

snrt_status snrt_step_imex_moments_f64(const snrt_mesh* m, const snrt_quad* q,
                                       const snrt_scatter* sc, const snrt_step_args_f64* a,
                                       const double* psi_in, double* psi_out, void* ws,
                                       size_t ws_bytes, void* stream) {
    g_last_error.clear();
    return imex_moments_common<double>("snrt_step_imex_moments_f64", m, q, sc, a, psi_in,
                                       psi_out, ws, ws_bytes, stream);
}

snrt_status snrt_step_imex_dense(const snrt_mesh* m, const snrt_quad* q, const snrt_scatter* sc,
                                 const snrt_step_args* a, const float* psi_in, float* psi_out,
                                 void* ws, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    return imex_dense_common<float>("snrt_step_imex_dense", m, q, sc, a, psi_in, psi_out, ws,
                                    ws_bytes, stream);
}

snrt_status snrt_step_imex_dense_f64(const snrt_mesh* m, const snrt_quad* q,
                                     const snrt_scatter* sc, const snrt_step_args_f64* a,
                                     const double* psi_in, double* psi_out, void* ws,
                                     size_t ws_bytes, void* stream) {
    g_last_error.clear();
    return imex_dense_common<double>("snrt_step_imex_dense_f64", m, q, sc, a, psi_in, psi_out,
                                     ws, ws_bytes, stream);
}

snrt_status snrt_scatter_apply(const snrt_mesh* m, const snrt_quad* q, const snrt_scatter* sc,
                               const float* psi, float* S, int32_t transpose, void* ws,
                               size_t ws_bytes, void* stream) {
    g_last_error.clear();
    SNRT_REQUIRE(m && q && sc, SNRT_E_ARG, "snrt_scatter_apply: NULL handle");
    SNRT_REQUIRE(sc->dense, SNRT_E_UNSUPPORTED,
                 "snrt_scatter_apply: needs a dense or moment scatter handle");
    SNRT_REQUIRE(sc->B.nq == q->nq, SNRT_E_SHAPE, "snrt_scatter_apply: scatter/quad nq differ");
    SNRT_REQUIRE(transpose == 0 || transpose == 1, SNRT_E_ARG, "snrt_scatter_apply: transpose is 0 or 1");
    SNRT_TRY(check_device(m->device, "snrt_scatter_apply"));
    if (m->nc == 0) return SNRT_OK;
    SNRT_REQUIRE(psi && S && aligned16(psi) && aligned16(S), SNRT_E_ARG,
                 "snrt_scatter_apply: NULL or misaligned array");
    const size_t bytes = (size_t)m->nc * q->nq * sizeof(float);
    SNRT_REQUIRE(!ranges_overlap(psi, bytes, S, bytes), SNRT_E_ALIAS, "snrt_scatter_apply: S aliases psi");
    // the workspace past the product itself: moments and FP16 row exponents
    const size_t need = (product_ws_elems(sc, m->nc) - (size_t)m->nc * q->nq) * sizeof(float);
    float* after = nullptr;
    if (need > 0) {
        SNRT_REQUIRE(ws && ws_bytes >= need && aligned16(ws), SNRT_E_ARG,
                     "snrt_scatter_apply: this handle needs a 16-byte aligned workspace of " +
                         std::to_string(need) + " bytes");
        SNRT_REQUIRE(!ranges_overlap(ws, need, psi, bytes) && !ranges_overlap(ws, need, S, bytes),
                     SNRT_E_ALIAS, "snrt_scatter_apply: workspace aliases psi or S");
        after = static_cast<float*>(ws);
    }
    hipError_t e = scatter_product32(sc, psi, S, m->nc, transpose != 0, after,
                                     static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SNRT_OK : hip_fail(e, "snrt_scatter_apply: launch");
}

// ------------------------------------------------------------------------------- reductions

snrt_status snrt_mass(const snrt_mesh* m, const snrt_quad* q, const float* psi, double* out,
                      void* stream) {
    g_last_error.clear();
    SNRT_REQUIRE(m && q && out, SNRT_E_ARG, "snrt_mass: NULL argument");
    SNRT_REQUIRE(psi || m->nc == 0, SNRT_E_ARG, "snrt_mass: NULL psi");
    SNRT_TRY(check_device(m->device, "snrt_mass"));
    hipError_t e = launch_mass(*m, *q, psi, out, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SNRT_OK : hip_fail(e, "snrt_mass: launch");
}

snrt_status snrt_scalar_flux(const snrt_mesh* m, const snrt_quad* q, const float* psi,
                             float* phi, void* stream) {
    g_last_error.clear();
    SNRT_REQUIRE(m && q, SNRT_E_ARG, "snrt_scalar_flux: NULL handle");
    SNRT_REQUIRE((psi && phi) || m->nc == 0, SNRT_E_ARG, "snrt_scalar_flux: NULL array");
    SNRT_TRY(check_device(m->device, "snrt_scalar_flux"));
    hipError_t e = launch_scalar_flux(*m, *q, psi, phi, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SNRT_OK : hip_fail(e, "snrt_scalar_flux: launch");
}

snrt_status snrt_dose_accumulate(const snrt_mesh* m, const snrt_quad* q, const float* psi,
                                 const float* inv_rho, double coeff, double* dose, void* stream) {
    g_last_error.clear();
    SNRT_REQUIRE(m && q, SNRT_E_ARG, "snrt_dose_accumulate: NULL handle");
    SNRT_REQUIRE((psi && dose) || m->nc == 0, SNRT_E_ARG, "snrt_dose_accumulate: NULL array");
    SNRT_REQUIRE(is_finite(coeff), SNRT_E_NONFINITE, "snrt_dose_accumulate: non-finite coeff");
    SNRT_TRY(check_device(m->device, "snrt_dose_accumulate"));
    hipError_t e = launch_dose(*m, *q, psi, inv_rho, coeff, dose, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SNRT_OK : hip_fail(e, "snrt_dose_accumulate: launch");
}

snrt_status snrt_dose_adjoint(const snrt_mesh* m, const snrt_quad* q, const float* inv_rho,
                              double coeff, const double* g_dose, float* lam, void* stream) {
    g_last_error.clear();
    SNRT_REQUIRE(m && q, SNRT_E_ARG, "snrt_dose_adjoint: NULL handle");
    SNRT_REQUIRE((g_dose && lam) || m->nc == 0, SNRT_E_ARG, "snrt_dose_adjoint: NULL array");
    SNRT_REQUIRE(is_finite(coeff), SNRT_E_NONFINITE, "snrt_dose_adjoint: non-finite coeff");
    SNRT_TRY(check_device(m->device, "snrt_dose_adjoint"));
    hipError_t e = launch_dose_adjoint(*m, *q, inv_rho, coeff, g_dose, lam,
                                       static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SNRT_OK : hip_fail(e, "snrt_dose_adjoint: launch");
}

snrt_status snrt_dose_density_grad(const snrt_mesh* m, const double* dose, const float* inv_rho,
                                   const double* g_dose, float* g_rho, void* stream) {
    g_last_error.clear();
    SNRT_REQUIRE(m, SNRT_E_ARG, "snrt_dose_density_grad: NULL mesh");
    SNRT_REQUIRE((dose && g_dose && g_rho) || m->nc == 0, SNRT_E_ARG,
                 "snrt_dose_density_grad: NULL array");
    SNRT_TRY(check_device(m->device, "snrt_dose_density_grad"));
    hipError_t e = launch_dose_density_grad(*m, dose, inv_rho, g_dose, g_rho,
                                            static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SNRT_OK : hip_fail(e, "snrt_dose_density_grad: launch");
}

snrt_status snrt_permute(const snrt_mesh* m, int32_t to_user, const void* in, void* out,
                         int64_t row_bytes, void* stream) {
    g_last_error.clear();
    SNRT_REQUIRE(m, SNRT_E_ARG, "snrt_permute: NULL mesh");
    SNRT_REQUIRE(to_user == 0 || to_user == 1, SNRT_E_ARG, "snrt_permute: direction must be 0 or 1");
    SNRT_REQUIRE(row_bytes > 0 && row_bytes % 4 == 0, SNRT_E_ARG,
                 "snrt_permute: row_bytes must be a positive multiple of 4");
    if (m->nc == 0) return SNRT_OK;
    SNRT_REQUIRE(in && out, SNRT_E_ARG, "snrt_permute: NULL array");
    SNRT_REQUIRE(((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 3u) == 0,
                 SNRT_E_ARG, "snrt_permute: arrays must be 4-byte aligned");
    const size_t bytes = (size_t)m->nc * row_bytes;
    SNRT_REQUIRE(!ranges_overlap(in, bytes, out, bytes), SNRT_E_ALIAS, "snrt_permute: out aliases in");
    SNRT_TRY(check_device(m->device, "snrt_permute"));
    hipError_t e = launch_permute(*m, to_user, in, out, row_bytes, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SNRT_OK : hip_fail(e, "snrt_permute: launch");
}

// ------------------------------------------------------------------- measurement helper

snrt_status snrt_stream_copy(const void* src, void* dst, int64_t bytes, void* stream) {
    g_last_error.clear();
    SNRT_REQUIRE(bytes >= 0 && bytes % 16 == 0, SNRT_E_ARG,
                 "snrt_stream_copy: bytes must be a non-negative multiple of 16");
    if (bytes == 0) return SNRT_OK;
    SNRT_REQUIRE(src && dst, SNRT_E_ARG, "snrt_stream_copy: NULL array");
    SNRT_REQUIRE(((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15u) == 0,
                 SNRT_E_ARG, "snrt_stream_copy: arrays must be 16-byte aligned");
    SNRT_REQUIRE(!ranges_overlap(src, (size_t)bytes, dst, (size_t)bytes), SNRT_E_ALIAS,
                 "snrt_stream_copy: dst overlaps src");
    hipError_t e = launch_stream_copy(src, dst, bytes, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SNRT_OK : hip_fail(e, "snrt_stream_copy: launch");
}

}  // extern "C"
