// Dense coupled path (pose-pair Hessian blocks and blocked Cholesky).
#include <hip/hip_runtime.h>

#include "ba.h"
#include "ba_internal.hpp"

namespace ba {

size_t dense_solve_workspace(int64_t n) { return 256; }

ba_status dense_prepare(Problem *P) {
    set_error("coupled mode not built yet");
    return BA_E_UNSUPPORTED;
}

ba_status dense_assemble(Problem *P, const double *poses, double *hess_out, bool use_lm, hipStream_t s) {
    set_error("coupled mode not built yet");
    return BA_E_UNSUPPORTED;
}

ba_status dense_solve(int64_t n, const double *A, const double *g, double mu, double *dx, int32_t *info, void *ws,
                      size_t ws_bytes, hipStream_t s) {
    set_error("coupled mode not built yet");
    return BA_E_UNSUPPORTED;
}

ba_status dense_lm_step(Problem *P, const double *poses, hipStream_t s) {
    set_error("coupled mode not built yet");
    return BA_E_UNSUPPORTED;
}

}  // namespace ba
