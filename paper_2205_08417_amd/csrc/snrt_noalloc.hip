// snrt_step_dose_noalloc: the fused dose step of snrt_step_dose for isotropic scattering,
// with the step's FP64 per-cell dose partials in a static device array of this library
// instead of a caller's workspace.  For callers that cannot allocate device memory (code
// under stream capture, serving loops, harnesses that forbid it): the call needs no
// workspace and allocates nothing.
//
// The array is file-scope __device__ memory, one copy per device, held until the process
// ends.  Its device address is looked up once per device (hipGetSymbolAddress, with that
// device current) and only that address is handed to kernels; the array's name is a host
// stand-in in host code and is never passed anywhere.  The kernels write every partial
// they later read, so nothing has to be cleared between calls; calls that overlap in time
// on one device share the array and race.
#include <mutex>
#include <string>

#include "snrt_internal.h"

namespace {

// One FP64 dose partial per cell (isotropic scattering: one work item per row).
constexpr int64_t kScratchDoubles = int64_t(1) << 20;   // 8 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array, looked up on first use.
snrt_status scratch_address(int dev, double** out) {
    *out = nullptr;
    if (dev < 0 || dev >= kMaxDevices) {
        snrt::set_error("snrt_step_dose_noalloc: device index out of range");
        return SNRT_E_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        // each device holds its own copy of the array: look it up with that device current
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
        void* p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur >= 0 && cur != dev) {
            hipError_t r = hipSetDevice(cur);
            if (e == hipSuccess) e = r;
        }
        if (e != hipSuccess || !p)
            return snrt::hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                  "snrt_step_dose_noalloc: scratch address");
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return SNRT_OK;
}

}  // namespace

extern "C" snrt_status snrt_step_dose_noalloc(const snrt_mesh* m, const snrt_quad* q,
                                              const snrt_scatter* sc, const snrt_step_args* a,
                                              const float* psi_in, float* psi_out,
                                              double coeff, double* dose, void* stream) {
    using namespace snrt;
    set_error("");
    const char* fn = "snrt_step_dose_noalloc";
    if (!m || !q || !sc || !a) {
        set_error(std::string(fn) + ": NULL handle or args");
        return SNRT_E_ARG;
    }
    if (sc->dense) {
        set_error(std::string(fn) + ": dense and moment scattering need the product workspace "
                  "(use snrt_step_dose)");
        return SNRT_E_UNSUPPORTED;
    }
    if (m->nc > kScratchDoubles) {
        set_error(std::string(fn) + ": " + std::to_string(m->nc) + " cells exceed the " +
                  std::to_string(kScratchDoubles) + " dose partials of the static scratch");
        return SNRT_E_UNSUPPORTED;
    }
    if (!is_finite(coeff)) {
        set_error(std::string(fn) + ": non-finite coeff");
        return SNRT_E_NONFINITE;
    }
    snrt_status s = check_step32(fn, m, q, sc, a, psi_in, psi_out, nullptr, 0);
    if (s != SNRT_OK) return s;
    if (m->nc == 0) return SNRT_OK;
    if (!dose) {
        set_error(std::string(fn) + ": NULL dose");
        return SNRT_E_ARG;
    }
    const size_t rows = (size_t)m->nc * q->nq * sizeof(float), db = (size_t)m->nc * sizeof(double);
    if (ranges_overlap(dose, db, psi_in, rows) || ranges_overlap(dose, db, psi_out, rows)) {
        set_error(std::string(fn) + ": dose aliases a state array");
        return SNRT_E_ALIAS;
    }
    double* part = nullptr;
    s = scratch_address(m->device, &part);
    if (s != SNRT_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = launch_step32(*m, *q, step_args32(a), psi_in, psi_out, nullptr, st, part);
    if (e == hipSuccess) e = launch_dose_fold(*m, part, 1, a->inv_rho, coeff, dose, st);
    return e == hipSuccess ? SNRT_OK : hip_fail(e, "snrt_step_dose_noalloc: launch");
}
