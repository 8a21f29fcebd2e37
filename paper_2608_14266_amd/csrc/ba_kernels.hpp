// Host-side launchers of the iteration kernels (internal to libba).
#pragma once
#include <hip/hip_runtime.h>

#include "ba_internal.hpp"

namespace ba {

// evaluation (ba_eval.hip)
void launch_vox(Problem *P, const double *poses, bool use_lm, bool trial, hipStream_t s);
void launch_window_cost(Problem *P, double *out, hipStream_t s);
// hess64: FP64 Hessian terms also in the precision form (the coupled form needs them)
void launch_pose_chunks(Problem *P, const double *poses, bool use_lm, hipStream_t s, bool hess64 = false);
void launch_pose_derivs(Problem *P, const double *poses, bool use_lm, double *g, double *H, hipStream_t s,
                        bool hess64 = false);
void launch_voxel_eig(Problem *P, double *out, hipStream_t s);

// LM (ba_lm.hip)
size_t solve_mm_workspace(int32_t n);
void launch_solve_mm_plain(int32_t n, const double *H, const double *g, double mu, double *dx, int32_t *info,
                           void *ws, hipStream_t s);
void launch_lm_reset(Problem *P, double mu0, double nu0, int32_t rejects0, const double *init, hipStream_t s);
void launch_lm_cost(Problem *P, hipStream_t s);
void launch_window_stats(Problem *P, double tol_g, hipStream_t s);
void launch_window_solve_mm(Problem *P, const double *poses, double tol_g, hipStream_t s);
DecideArgs decide_args(Problem *P, double *trace, int it, double *poses, int max_rejects);
void launch_decide(Problem *P, double *trace, int it, double *poses, hipStream_t s, int max_rejects);
void launch_commit(Problem *P, double *poses, hipStream_t s);

}  // namespace ba
