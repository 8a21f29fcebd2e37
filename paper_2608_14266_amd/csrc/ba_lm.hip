// Increment solve, SE(3) update and Levenberg-Marquardt control, all on the
// device so that an iteration needs no host round trip (the paper runs LM
// sequentially on the CPU, Fig. 1; PredResReduction and Adjust of Alg. 2 are
// declared there but not printed).
//
//  k_solve_mm   — Alg. 2 Solver: one thread per scan factors the 6x6
//                 H_jj + mu D_jj by LDL^T, solves for dx_j, forms the trial
//                 pose T_j (+) dx_j and its share of the predicted reduction.
//  k_window_stats / k_decide — per-window gradient norm and damping floor;
//                 gain ratio, damping update and commit of accepted poses.
#include <hip/hip_runtime.h>

#include "ba.h"
#include "ba_device.hpp"
#include "ba_internal.hpp"
#include "ba_kernels.hpp"
#include "ba_decide.hpp"

namespace ba {

// LDL^T solve of a 6x6 symmetric positive definite system held in registers.
// Returns 0, or the 1-based index of the first non-positive pivot.
__device__ __forceinline__ int ldlt6(double A[6][6], const double b[6], double x[6]) {
    double d[6];
#pragma unroll
    for (int j = 0; j < 6; j++) {
        double s = A[j][j];
#pragma unroll
        for (int k = 0; k < j; k++) s -= A[j][k] * A[j][k] * d[k];
        if (!(s > 0.0)) return j + 1;
        d[j] = s;
        const double inv = 1.0 / s;
#pragma unroll
        for (int i = j + 1; i < 6; i++) {
            double t = A[i][j];
#pragma unroll
            for (int k = 0; k < j; k++) t -= A[i][k] * A[j][k] * d[k];
            A[i][j] = t * inv;  // L[i][j]
        }
    }
    double y[6];
#pragma unroll
    for (int i = 0; i < 6; i++) {
        double t = b[i];
#pragma unroll
        for (int k = 0; k < i; k++) t -= A[i][k] * y[k];
        y[i] = t;
    }
#pragma unroll
    for (int i = 0; i < 6; i++) y[i] /= d[i];
#pragma unroll
    for (int i = 5; i >= 0; i--) {
        double t = y[i];
#pragma unroll
        for (int k = i + 1; k < 6; k++) t -= A[k][i] * x[k];
        x[i] = t;
    }
    return 0;
}

// Damped 6x6 solve of one scan; returns info (0 ok).  q_out = -(g dx + dx H dx / 2).
__device__ __forceinline__ int solve_pose(const double *__restrict__ h, const double *__restrict__ gj, double mu,
                                          double floor_, double *dxj, double &q_out) {
    double A[6][6], b[6], x[6];
#pragma unroll
    for (int r = 0; r < 6; r++) {
#pragma unroll
        for (int c = 0; c < 6; c++) A[r][c] = h[6 * r + c];
        const double hk = A[r][r];
        A[r][r] += mu * (hk > floor_ ? hk : floor_);
        b[r] = -gj[r];
    }
    const int info = ldlt6(A, b, x);
    if (info) {
#pragma unroll
        for (int r = 0; r < 6; r++) dxj[r] = 0.0;
        q_out = 0.0;
        return info;
    }
    double gdx = 0.0, dhd = 0.0;
#pragma unroll
    for (int r = 0; r < 6; r++) {
        gdx += gj[r] * x[r];
        double hr = 0.0;
#pragma unroll
        for (int c = 0; c < 6; c++) hr += h[6 * r + c] * x[c];
        dhd += x[r] * hr;
        dxj[r] = x[r];
    }
    q_out = -(gdx + 0.5 * dhd);
    return 0;
}

__global__ void k_lm_reset(int32_t W, LMState *__restrict__ lm, double mu0, double nu0,
                           const int32_t *__restrict__ win_group_ptr) {
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= W) return;
    LMState s;
    s.mu = mu0; s.nu = nu0; s.cost = 0.0; s.cost_trial = 0.0; s.q = 0.0; s.rho = 0.0;
    s.gnorm = 0.0; s.maxdiag = 0.0; s.cost0 = 0.0;
    s.accepted = 0; s.need_eval = 1; s.info = 0;
    s.done = (win_group_ptr[w + 1] == win_group_ptr[w]) ? 1 : 0;   // a window without voxels has nothing to do
    s.iters = 0; s.n_accepted = 0; s.cur = 0; s.rejects = 0;
    lm[w] = s;
}

// block per window: cost at the current poses from the group residuals (the
// same summation order as the trial cost of the decision kernel)
__global__ __launch_bounds__(DECIDE_THREADS) void k_lm_cost(int32_t W, const int32_t *__restrict__ win_group_ptr,
                                                            const double *__restrict__ wave_cost,
                                                            LMState *__restrict__ lm) {
    __shared__ double red[DECIDE_THREADS / 64];
    const int w = blockIdx.x;
    if (w >= W) return;
    const double c = window_cost_sum(win_group_ptr[w], win_group_ptr[w + 1], wave_cost, red);
    if (threadIdx.x == 0) {
        lm[w].cost = c;
        lm[w].cost0 = c;
    }
}

// block per window: ||g|| and max diag(H) at freshly evaluated poses; convergence test.
// Gradient norm and largest Hessian diagonal of every window whose
// derivatives are fresh, in the order the fused MM solve forms them (per pose,
// then the wave totals in wave order).
__global__ __launch_bounds__(1024) void k_window_stats(int32_t W, const int32_t *__restrict__ win_pose_ptr,
                                                       const double *__restrict__ g, const double *__restrict__ H,
                                                       LMState *__restrict__ lm, double tol_g) {
    constexpr int NW = 1024 / 64;
    __shared__ double red[NW];
    const int w = blockIdx.x;
    if (w >= W) return;
    LMState &st = lm[w];
    if (st.done || !st.need_eval) return;
    double s = 0.0, m = 0.0;
    const int p0 = win_pose_ptr[w], p1 = win_pose_ptr[w + 1];
    for (int j = p0 + threadIdx.x; j < p1; j += 1024) {
#pragma unroll
        for (int k = 0; k < 6; k++) {
            const double gk = g[6LL * j + k];
            s = fma(gk, gk, s);
            m = fmax(m, H[36LL * j + 7 * k]);
        }
    }
    s = block_sum<NW>(s, red);
    m = block_max<NW>(m, red);
    if (threadIdx.x == 0) {
        st.gnorm = sqrt(s);
        st.maxdiag = m;
        st.need_eval = 0;
        if (tol_g > 0.0 && st.gnorm < tol_g) {
            st.done = 1;
            st.accepted = 0;
        }
    }
}

__global__ void k_solve_mm_lm(int32_t n_poses, const int32_t *__restrict__ pose_window,
                              const int32_t *__restrict__ win_pose_ptr, const LMState *__restrict__ lm,
                              const double *__restrict__ H, const double *__restrict__ g,
                              const double *__restrict__ poses, double *__restrict__ dx, double *__restrict__ pose_q,
                              int32_t *__restrict__ pose_info, double *__restrict__ poses_trial) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_poses) return;
    const int w = pose_window[j];
    const LMState &st = lm[w];
    if (st.done) return;
    double q;
    const int info = solve_pose(H + 36LL * j, g + 6LL * j, st.mu, 1e-12 * st.maxdiag, dx + 6LL * j, q);
    pose_q[j] = q;
    pose_info[j] = info ? 6 * (j - win_pose_ptr[w]) + info : 0;
    pose_plus(poses + 12LL * j, dx + 6LL * j, poses_trial + 12LL * j);
}

// block per window: predicted reduction, trial cost, gain ratio, damping update.
__global__ __launch_bounds__(DECIDE_THREADS) void k_decide(DecideArgs da) {
    if ((int)blockIdx.x >= da.W) return;
    decide_window(blockIdx.x, da);
}

__global__ void k_commit(int32_t n_poses, const int32_t *__restrict__ pose_window, const LMState *__restrict__ lm,
                         const double *__restrict__ poses_trial, double *__restrict__ poses) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 12LL * n_poses) return;
    const int j = (int)(i / 12);
    const LMState &st = lm[pose_window[j]];
    if (!st.done && st.accepted) poses[i] = poses_trial[i];
}

// One 512-thread block per window: when the derivatives are fresh, the
// window's gradient norm and largest Hessian diagonal (per thread over poses
// p0 + t, p0 + t + 512, ..., then the wave totals in wave order) and the
// convergence test; then every pose's damped 6x6 system is solved and the
// trial pose T (+) dx formed.  Windows of more than SPLIT_SOLVE_POSES poses
// take two launches instead, the same statistics in the same order
// (k_window_stats_mm) and one thread per pose over the whole grid
// (k_solve_mm_lm), so the results do not depend on which form runs.
static constexpr int WSOLVE_THREADS = 512;
static constexpr int SPLIT_SOLVE_POSES = 1024;

// Returns whether the window is finished (block-uniform).  `red` holds
// 2 * WSOLVE_THREADS / 64 doubles.
__device__ __forceinline__ bool window_fresh_stats(LMState &st, const double *__restrict__ g,
                                                   const double *__restrict__ H, int p0, int p1, double tol_g,
                                                   double *red, int *s_done) {
    constexpr int NW = WSOLVE_THREADS / 64;
    if (!st.need_eval) return false;
    double gs = 0.0, mx = 0.0;
    for (int j = p0 + threadIdx.x; j < p1; j += WSOLVE_THREADS) {
#pragma unroll
        for (int k = 0; k < 6; k++) {
            const double gk = g[6LL * j + k];
            gs = fma(gk, gk, gs);
            mx = fmax(mx, H[36LL * j + 7 * k]);
        }
    }
    block_sum_max<NW>(gs, mx, red, red + NW);
    if (threadIdx.x == 0) {
        st.gnorm = sqrt(gs);
        st.maxdiag = mx;
        st.need_eval = 0;
        if (tol_g > 0.0 && st.gnorm < tol_g) {
            st.done = 1;
            st.accepted = 0;
        }
        *s_done = st.done;
    }
    __syncthreads();
    return *s_done != 0;
}

__global__ __launch_bounds__(WSOLVE_THREADS) void k_window_solve_mm(
    int32_t W, const int32_t *__restrict__ win_pose_ptr, LMState *__restrict__ lm, const double *__restrict__ g,
    const double *__restrict__ H, const double *__restrict__ poses, double *__restrict__ dx,
    double *__restrict__ pose_q, int32_t *__restrict__ pose_info, double *__restrict__ poses_trial, double tol_g) {
    __shared__ double red[2 * (WSOLVE_THREADS / 64)];
    __shared__ int s_done;
    const int w = blockIdx.x;
    if (w >= W) return;
    LMState &st = lm[w];
    if (st.done) return;
    const int p0 = win_pose_ptr[w], p1 = win_pose_ptr[w + 1];
    if (window_fresh_stats(st, g, H, p0, p1, tol_g, red, &s_done)) return;
    const double mu = st.mu, fl = 1e-12 * st.maxdiag;
    for (int j = p0 + threadIdx.x; j < p1; j += WSOLVE_THREADS) {
        double q;
        const int info = solve_pose(H + 36LL * j, g + 6LL * j, mu, fl, dx + 6LL * j, q);
        pose_q[j] = q;
        pose_info[j] = info ? 6 * (j - p0) + info : 0;
        pose_plus(poses + 12LL * j, dx + 6LL * j, poses_trial + 12LL * j);
    }
}

__global__ __launch_bounds__(WSOLVE_THREADS) void k_window_stats_mm(int32_t W,
                                                                    const int32_t *__restrict__ win_pose_ptr,
                                                                    LMState *__restrict__ lm,
                                                                    const double *__restrict__ g,
                                                                    const double *__restrict__ H, double tol_g) {
    __shared__ double red[2 * (WSOLVE_THREADS / 64)];
    __shared__ int s_done;
    const int w = blockIdx.x;
    if (w >= W) return;
    LMState &st = lm[w];
    if (st.done) return;
    (void)window_fresh_stats(st, g, H, win_pose_ptr[w], win_pose_ptr[w + 1], tol_g, red, &s_done);
}

void launch_window_solve_mm(Problem *P, const double *poses, double tol_g, hipStream_t s) {
    int32_t widest = 0;
    for (int32_t w = 0; w < P->n_windows; w++)
        widest = std::max(widest, P->h_win_pose_ptr[w + 1] - P->h_win_pose_ptr[w]);
    ProfScope prof("k_window_solve_mm", s);
    if (widest > SPLIT_SOLVE_POSES) {
        hipLaunchKernelGGL(k_window_stats_mm, dim3(P->n_windows), dim3(WSOLVE_THREADS), 0, s, P->n_windows,
                           P->win_pose_ptr, P->lm, P->g, P->H, tol_g);
        hipLaunchKernelGGL(k_solve_mm_lm, dim3((unsigned)((P->n_poses + 255) / 256)), dim3(256), 0, s, P->n_poses,
                           P->pose_window, P->win_pose_ptr, P->lm, P->H, P->g, poses, P->dx, P->pose_q, P->pose_info,
                           P->poses_trial);
        return;
    }
    hipLaunchKernelGGL(k_window_solve_mm, dim3(P->n_windows), dim3(WSOLVE_THREADS), 0, s, P->n_windows,
                       P->win_pose_ptr, P->lm, P->g, P->H, poses, P->dx, P->pose_q, P->pose_info, P->poses_trial,
                       tol_g);
}

// ---------------------------------------------------------------- standalone MM solve
__global__ __launch_bounds__(256) void k_maxdiag_mm(int32_t n, const double *__restrict__ H,
                                                    double *__restrict__ out) {
    __shared__ double rm[256];
    double m = 0.0;
    for (int i = threadIdx.x; i < 6 * n; i += 256) m = fmax(m, H[36LL * (i / 6) + 7 * (i % 6)]);
    rm[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) rm[threadIdx.x] = fmax(rm[threadIdx.x], rm[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = rm[0];
}

__global__ void k_solve_mm_plain(int32_t n, const double *__restrict__ H, const double *__restrict__ g, double mu,
                                 const double *__restrict__ maxdiag, double *__restrict__ dx,
                                 int32_t *__restrict__ infos) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double q;
    const int info = solve_pose(H + 36LL * j, g + 6LL * j, mu, 1e-12 * maxdiag[0], dx + 6LL * j, q);
    infos[j] = info ? 6 * j + info : 0;
}

__global__ __launch_bounds__(256) void k_solve_finish(int32_t n, const int32_t *__restrict__ infos,
                                                      double *__restrict__ dx, int32_t *__restrict__ info) {
    __shared__ int ri[256];
    int m = 0x7fffffff;
    for (int j = threadIdx.x; j < n; j += 256)
        if (infos[j]) m = min(m, infos[j]);
    ri[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) ri[threadIdx.x] = min(ri[threadIdx.x], ri[threadIdx.x + o]);
        __syncthreads();
    }
    const int r = (ri[0] == 0x7fffffff) ? 0 : ri[0];
    if (r)
        for (int i = threadIdx.x; i < 6 * n; i += 256) dx[i] = 0.0;
    if (threadIdx.x == 0) *info = r;
}

static inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

size_t solve_mm_workspace(int32_t n) { return align_up(sizeof(double), 256) + sizeof(int32_t) * (size_t)n + 256; }

void launch_solve_mm_plain(int32_t n, const double *H, const double *g, double mu, double *dx, int32_t *info,
                           void *ws, hipStream_t s) {
    double *md = (double *)ws;
    int32_t *infos = (int32_t *)((char *)ws + align_up(sizeof(double), 256));
    hipLaunchKernelGGL(k_maxdiag_mm, dim3(1), dim3(256), 0, s, n, H, md);
    hipLaunchKernelGGL(k_solve_mm_plain, dim3(nblk(n)), dim3(256), 0, s, n, H, g, mu, md, dx, infos);
    hipLaunchKernelGGL(k_solve_finish, dim3(1), dim3(256), 0, s, n, infos, dx, info);
}

void launch_lm_reset(Problem *P, double mu0, double nu0, hipStream_t s) {
    hipLaunchKernelGGL(k_lm_reset, dim3(nblk(P->n_windows)), dim3(256), 0, s, P->n_windows, P->lm, mu0, nu0,
                       P->win_group_ptr);
}

void launch_lm_cost(Problem *P, hipStream_t s) {
    hipLaunchKernelGGL(k_lm_cost, dim3(P->n_windows), dim3(DECIDE_THREADS), 0, s, P->n_windows, P->win_group_ptr,
                       P->wave_cost, P->lm);
}

void launch_window_stats(Problem *P, double tol_g, hipStream_t s) {
    hipLaunchKernelGGL(k_window_stats, dim3(P->n_windows), dim3(1024), 0, s, P->n_windows, P->win_pose_ptr, P->g,
                       P->H, P->lm, tol_g);
}

DecideArgs decide_args(Problem *P, double *trace, int it, double *poses, int max_rejects) {
    DecideArgs da;
    da.max_rejects = max_rejects;
    da.W = P->n_windows;
    da.win_pose_ptr = P->win_pose_ptr;
    da.win_group_ptr = P->win_group_ptr;
    da.pose_q = P->pose_q;
    da.pose_info = P->pose_info;
    da.group_cost = P->wave_cost;
    da.lm = P->lm;
    da.trace = trace;
    da.it = it;
    da.poses_trial = P->poses_trial;
    da.poses = poses;
    return da;
}

void launch_decide(Problem *P, double *trace, int it, double *poses, hipStream_t s, int max_rejects) {
    DecideArgs da = decide_args(P, trace, it, poses, max_rejects);
    ProfScope prof("k_decide", s);
    hipLaunchKernelGGL(k_decide, dim3(P->n_windows), dim3(DECIDE_THREADS), 0, s, da);
}

void launch_commit(Problem *P, double *poses, hipStream_t s) {
    hipLaunchKernelGGL(k_commit, dim3(nblk(12LL * P->n_poses)), dim3(256), 0, s, P->n_poses, P->pose_window, P->lm,
                       P->poses_trial, poses);
}

}  // namespace ba
