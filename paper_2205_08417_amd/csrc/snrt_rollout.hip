// Multi-step drivers of the C ABI: a forward rollout of explicit steps with checkpoints, and
// the reverse pass over it (segment recompute from each checkpoint, then the transposed steps
// backwards).  They only sequence the library's own step, dose and adjoint entry points on
// one stream, so the host issues each launch as fast as the device retires the previous one
// and no per-step work is left to an interpreter.  Time loop: Alg. "Execution of the solver"
// with one Runge-Kutta stage (explicit Euler).
#include <algorithm>
#include <string>
#include <type_traits>
#include <vector>

#include "snrt_internal.h"

using namespace snrt;

#define SNRT_REQUIRE(cond, code, msg) \
    do {                              \
        if (!(cond)) {                \
            set_error(msg);           \
            return code;              \
        }                             \
    } while (0)

namespace {

template <typename T> struct Api;
template <> struct Api<float> {
    using Args = snrt_step_args;
    static snrt_status step(const snrt_mesh* m, const snrt_quad* q, const snrt_scatter* sc,
                            const Args* a, const float* in, float* out, void* ws, size_t wsb,
                            void* st) {
        return snrt_step(m, q, sc, a, in, out, ws, wsb, st);
    }
    // gradients accumulate in FP64 across the steps of a reverse pass; da: the dose
    // functional's term, added to the transposed step's output rows
    static snrt_status adjoint(const snrt_mesh* m, const snrt_quad* q, const snrt_scatter* sc,
                               const Args* a, const float* psi, const float* l1, float* l0,
                               double* gt, double* gs, double* gr, void* ws, size_t wsb,
                               void* st, const DoseAdj& da = DoseAdj()) {
        return step_adjoint32_acc64(m, q, sc, a, psi, l1, l0, gt, gs, gr, ws, wsb, st, da);
    }
};
template <> struct Api<double> {
    using Args = snrt_step_args_f64;
    static snrt_status step(const snrt_mesh* m, const snrt_quad* q, const snrt_scatter* sc,
                            const Args* a, const double* in, double* out, void* ws, size_t wsb,
                            void* st) {
        return snrt_step_f64(m, q, sc, a, in, out, ws, wsb, st);
    }
    static snrt_status adjoint(const snrt_mesh* m, const snrt_quad* q, const snrt_scatter* sc,
                               const Args* a, const double* psi, const double* l1, double* l0,
                               double* gt, double* gs, double* gr, void* ws, size_t wsb,
                               void* st) {
        return snrt_step_adjoint_f64(m, q, sc, a, psi, l1, l0, gt, gs, gr, ws, wsb, st);
    }
};

// The step arguments of step n: args with the schedule's per-step scalars substituted.
template <typename Args>
Args step_n(const Args& a, const snrt_schedule* s, int64_t n) {
    Args r = a;
    if (s) {
        if (s->alpha_t) r.alpha_t = s->alpha_t[n];
        if (s->alpha_s) r.alpha_s = s->alpha_s[n];
        if (s->inflow_scale) r.inflow_scale = s->inflow_scale[n];
    }
    return r;
}

snrt_status copy_state(void* dst, const void* src, size_t bytes, hipStream_t st,
                       const char* fn) {
    if (dst == src || bytes == 0) return SNRT_OK;
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st);
    return e == hipSuccess ? SNRT_OK : hip_fail(e, fn);
}

template <typename T>
snrt_status rollout_t(const char* fn, const snrt_mesh* m, const snrt_quad* q,
                      const snrt_scatter* sc, const typename Api<T>::Args* a,
                      const snrt_schedule* sched, int64_t nsteps, T* psi, T* tmp, T* ckpt,
                      int32_t ckpt_every, double* dose, void* ws, size_t ws_bytes,
                      void* stream) {
    SNRT_REQUIRE(m && q && sc && a, SNRT_E_ARG, std::string(fn) + ": NULL handle or args");
    SNRT_REQUIRE(nsteps >= 0, SNRT_E_ARG, std::string(fn) + ": nsteps < 0");
    SNRT_REQUIRE(!ckpt || ckpt_every >= 1, SNRT_E_ARG,
                 std::string(fn) + ": ckpt_every must be >= 1 with checkpoints");
    if (nsteps == 0 || m->nc == 0) return SNRT_OK;
    SNRT_REQUIRE(psi && tmp, SNRT_E_ARG, std::string(fn) + ": NULL state buffer");
    SNRT_REQUIRE(!dose || (sched && sched->dose_coeff), SNRT_E_ARG,
                 std::string(fn) + ": a dose needs the schedule's dose_coeff");
    const size_t elems = (size_t)m->nc * q->nq, bytes = elems * sizeof(T);
    SNRT_REQUIRE(!ranges_overlap(psi, bytes, tmp, bytes), SNRT_E_ALIAS,
                 std::string(fn) + ": tmp overlaps psi");
    const int64_t nck = ckpt ? (nsteps + ckpt_every - 1) / ckpt_every : 0;
    if (ckpt) {
        const size_t cb = (size_t)nck * bytes;
        SNRT_REQUIRE(!ranges_overlap(ckpt, cb, psi, bytes) && !ranges_overlap(ckpt, cb, tmp, bytes),
                     SNRT_E_ALIAS, std::string(fn) + ": checkpoints overlap a state buffer");
    }
    // Where each state lives: psi^N in psi, checkpointed states in their slot (the step
    // before writes them there directly), the others alternating between psi and tmp so
    // that no step reads and writes the same buffer.
    std::vector<T*> buf((size_t)nsteps + 1);
    buf[nsteps] = psi;
    for (int64_t n = nsteps - 1; n >= 0; --n) {
        if (ckpt && n % ckpt_every == 0)
            buf[n] = ckpt + (size_t)(n / ckpt_every) * elems;
        else
            buf[n] = buf[n + 1] == psi ? tmp : psi;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    snrt_status s = copy_state(buf[0], psi, bytes, st, fn);
    for (int64_t n = 0; n < nsteps && s == SNRT_OK; ++n) {
        const auto an = step_n(*a, sched, n);
        if constexpr (std::is_same<T, float>::value) {
            if (dose) {
                s = snrt_step_dose(m, q, sc, &an, buf[n], buf[n + 1], sched->dose_coeff[n], dose,
                                   ws, ws_bytes, stream);
                continue;
            }
        }
        s = Api<T>::step(m, q, sc, &an, buf[n], buf[n + 1], ws, ws_bytes, stream);
    }
    return s;
}

template <typename T>
snrt_status rollout_adjoint_t(const char* fn, const snrt_mesh* m, const snrt_quad* q,
                              const snrt_scatter* sc, const typename Api<T>::Args* a,
                              const snrt_schedule* sched, int64_t nsteps, const T* ckpt,
                              int32_t ckpt_every, T* seg, T* lam, T* tmp, double* g_t,
                              double* g_s, double* g_r, const double* g_dose,
                              const double* dose, void* ws, size_t ws_bytes, void* stream) {
    SNRT_REQUIRE(m && q && sc && a, SNRT_E_ARG, std::string(fn) + ": NULL handle or args");
    SNRT_REQUIRE(nsteps >= 0, SNRT_E_ARG, std::string(fn) + ": nsteps < 0");
    SNRT_REQUIRE(ckpt_every >= 1, SNRT_E_ARG, std::string(fn) + ": ckpt_every must be >= 1");
    if (nsteps == 0 || m->nc == 0) return SNRT_OK;
    SNRT_REQUIRE(ckpt && lam && tmp, SNRT_E_ARG, std::string(fn) + ": NULL state buffer");
    SNRT_REQUIRE(ckpt_every == 1 || seg, SNRT_E_ARG,
                 std::string(fn) + ": ckpt_every > 1 needs the segment buffer");
    SNRT_REQUIRE(!g_dose || (sched && sched->dose_coeff), SNRT_E_ARG,
                 std::string(fn) + ": g_dose needs the schedule's dose_coeff");
    const size_t elems = (size_t)m->nc * q->nq, bytes = elems * sizeof(T);
    const int64_t nck = (nsteps + ckpt_every - 1) / ckpt_every;
    const size_t cb = (size_t)nck * bytes, sb = (size_t)(ckpt_every - 1) * bytes;
    SNRT_REQUIRE(!ranges_overlap(lam, bytes, tmp, bytes) && !ranges_overlap(lam, bytes, ckpt, cb) &&
                     !ranges_overlap(tmp, bytes, ckpt, cb),
                 SNRT_E_ALIAS, std::string(fn) + ": lam, tmp and the checkpoints must be disjoint");
    if (seg && sb)
        SNRT_REQUIRE(!ranges_overlap(seg, sb, lam, bytes) && !ranges_overlap(seg, sb, tmp, bytes) &&
                         !ranges_overlap(seg, sb, ckpt, cb),
                     SNRT_E_ALIAS, std::string(fn) + ": seg overlaps another buffer");
    hipStream_t st = static_cast<hipStream_t>(stream);
    T* pl = lam;
    T* pn = tmp;
    std::vector<const T*> states((size_t)ckpt_every);
    snrt_status s = SNRT_OK;
    for (int64_t k = nck - 1; k >= 0 && s == SNRT_OK; --k) {
        const int64_t n0 = k * ckpt_every;
        const int64_t L = std::min<int64_t>(ckpt_every, nsteps - n0);
        states[0] = ckpt + (size_t)k * elems;
        for (int64_t i = 1; i < L; ++i) states[i] = seg + (size_t)(i - 1) * elems;
        for (int64_t i = 0; i + 1 < L && s == SNRT_OK; ++i) {   // recompute the segment
            const auto an = step_n(*a, sched, n0 + i);
            s = Api<T>::step(m, q, sc, &an, states[i], const_cast<T*>(states[i + 1]), ws,
                             ws_bytes, stream);
        }
        for (int64_t i = L - 1; i >= 0 && s == SNRT_OK; --i) {
            const int64_t n = n0 + i;
            const auto an = step_n(*a, sched, n);
            if constexpr (std::is_same<T, float>::value) {
                // the dose functional's term rides on the transposed step's output (one pass
                // over lam instead of two); SNRT_STEP_FUSED=0 keeps it a pass of its own
                DoseAdj da;
                const bool fuse = g_dose && tune().step_fused;
                if (fuse) {
                    da.w = q->tab64 + 2 * (int64_t)q->nq;
                    da.coeff = sched->dose_coeff[n];
                    da.g_dose = g_dose;
                }
                s = Api<T>::adjoint(m, q, sc, &an, states[i], pl, pn, g_t, g_s, g_r, ws,
                                    ws_bytes, stream, da);
                if (s == SNRT_OK && g_dose && !fuse)
                    s = snrt_dose_adjoint(m, q, a->inv_rho, sched->dose_coeff[n], g_dose, pn,
                                          stream);
            } else {
                s = Api<T>::adjoint(m, q, sc, &an, states[i], pl, pn, g_t, g_s, g_r, ws,
                                    ws_bytes, stream);
            }
            std::swap(pl, pn);
        }
    }
    if (s == SNRT_OK) s = copy_state(lam, pl, bytes, st, fn);
    if constexpr (std::is_same<T, float>::value) {
        // the explicit density derivative of the dose, -D_i (1/rho_i) dJ/dD_i
        if (s == SNRT_OK && g_dose && dose && g_r) {
            hipError_t e = launch_dose_density_grad64(*m, dose, a->inv_rho, g_dose, g_r, st);
            if (e != hipSuccess) s = hip_fail(e, fn);
        }
    }
    return s;
}

}  // namespace

extern "C" {

snrt_status snrt_rollout(const snrt_mesh* m, const snrt_quad* q, const snrt_scatter* sc,
                         const snrt_step_args* a, const snrt_schedule* sched, int64_t nsteps,
                         float* psi, float* tmp, float* ckpt, int32_t ckpt_every, double* dose,
                         void* ws, size_t ws_bytes, void* stream) {
    set_error("");
    return rollout_t<float>("snrt_rollout", m, q, sc, a, sched, nsteps, psi, tmp, ckpt,
                            ckpt_every, dose, ws, ws_bytes, stream);
}

snrt_status snrt_rollout_f64(const snrt_mesh* m, const snrt_quad* q, const snrt_scatter* sc,
                             const snrt_step_args_f64* a, const snrt_schedule* sched,
                             int64_t nsteps, double* psi, double* tmp, double* ckpt,
                             int32_t ckpt_every, void* ws, size_t ws_bytes, void* stream) {
    set_error("");
    return rollout_t<double>("snrt_rollout_f64", m, q, sc, a, sched, nsteps, psi, tmp, ckpt,
                             ckpt_every, nullptr, ws, ws_bytes, stream);
}

snrt_status snrt_rollout_adjoint(const snrt_mesh* m, const snrt_quad* q, const snrt_scatter* sc,
                                 const snrt_step_args* a, const snrt_schedule* sched,
                                 int64_t nsteps, const float* ckpt, int32_t ckpt_every,
                                 float* seg, float* lam, float* tmp, double* g_sigma_t,
                                 double* g_sigma_s, double* g_rho, const double* g_dose,
                                 const double* dose, void* ws, size_t ws_bytes, void* stream) {
    set_error("");
    return rollout_adjoint_t<float>("snrt_rollout_adjoint", m, q, sc, a, sched, nsteps, ckpt,
                                    ckpt_every, seg, lam, tmp, g_sigma_t, g_sigma_s, g_rho,
                                    g_dose, dose, ws, ws_bytes, stream);
}

snrt_status snrt_rollout_adjoint_f64(const snrt_mesh* m, const snrt_quad* q,
                                     const snrt_scatter* sc, const snrt_step_args_f64* a,
                                     const snrt_schedule* sched, int64_t nsteps,
                                     const double* ckpt, int32_t ckpt_every, double* seg,
                                     double* lam, double* tmp, double* g_sigma_t,
                                     double* g_sigma_s, double* g_rho, void* ws, size_t ws_bytes,
                                     void* stream) {
    set_error("");
    return rollout_adjoint_t<double>("snrt_rollout_adjoint_f64", m, q, sc, a, sched, nsteps, ckpt,
                                     ckpt_every, seg, lam, tmp, g_sigma_t, g_sigma_s, g_rho,
                                     nullptr, nullptr, ws, ws_bytes, stream);
}

}  // extern "C"
