// Allocation-free damped increment solve: ba_solve_increment with its
// workspace taken from a static device array instead of the caller, for
// callers that cannot allocate device memory (see include/ba.h).
//
// `scratch` below is a file-scope device array.  In host code its name is a
// host-side stand-in, not a device address: the device address differs per
// GPU and is obtained once per device with hipGetSymbolAddress (with that
// device current) and kept in g_scratch[]; only that pointer is ever handed
// to kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "ba.h"
#include "ba_internal.hpp"
#include "ba_kernels.hpp"

namespace ba {

size_t dense_solve_workspace(int64_t n);
ba_status dense_solve(int64_t n, const double *A, const double *g, double mu, double *dx, int32_t *info, void *ws,
                      size_t ws_bytes, hipStream_t s);

static __device__ __align__(256) unsigned char scratch[BA_STATIC_SCRATCH_BYTES];

static constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch[MAX_DEVICES] = {};

// Device address of this GPU's copy of `scratch` (looked up on the first call
// on the device, with that device current).
static ba_status scratch_ptr(void **out) {
    int dev = -1;
    BA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) {
        set_error("device %d out of range of the static scratch table", dev);
        return BA_E_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            set_error("hipGetSymbolAddress of the static scratch failed: %s", hipGetErrorString(e));
            return BA_E_HIP;
        }
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return BA_OK;
}

}  // namespace ba

using namespace ba;

extern "C" ba_status ba_solve_increment_noalloc(int32_t mode, int32_t n_scans, const double *hess,
                                                const double *grad, double mu, double *dx, int32_t *info,
                                                hipStream_t stream) {
    if (mode != BA_MODE_MM && mode != BA_MODE_COUPLED && mode != BA_MODE_EXACT) {
        set_error("unknown mode %d", mode);
        return BA_E_UNSUPPORTED;
    }
    if (n_scans < 1 || !hess || !grad || !dx || !info || !(mu >= 0.0) || !std::isfinite(mu)) {
        set_error("invalid argument to ba_solve_increment_noalloc");
        return BA_E_ARG;
    }
    const size_t need = ba_solve_increment_workspace(mode, n_scans);
    if (need > (size_t)BA_STATIC_SCRATCH_BYTES) {
        set_error("the solve of %d scans needs %zu bytes of scratch; the static scratch holds %zu", n_scans, need,
                  (size_t)BA_STATIC_SCRATCH_BYTES);
        return BA_E_WORKSPACE;
    }
    void *ws = nullptr;
    BA_TRY(scratch_ptr(&ws));
    // the solve's kernels write every scratch word they later read (nothing
    // needs to start at zero): the same launches as ba_solve_increment
    if (mode == BA_MODE_MM) {
        launch_solve_mm_plain(n_scans, hess, grad, mu, dx, info, ws, stream);
        BA_HIP(hipGetLastError());
        return BA_OK;
    }
    return dense_solve(6LL * n_scans, hess, grad, mu, dx, info, ws, need, stream);
}
