// Increment solve, SE(3) update and Levenberg-Marquardt control, all on the
// device so that an iteration needs no host round trip (the paper runs LM
// sequentially on the CPU, Fig. 1; PredResReduction and Adjust of Alg. 2 are
// declared there but not printed).
//
//  k_window_solve_mm — Alg. 2 Solver: per-window gradient norm and damping
//                 floor, then one thread per scan factors the 6x6
//                 H_jj + mu D_jj by LDL^T, solves for dx_j, forms the trial
//                 pose T_j (+) dx_j and its share of the predicted reduction.
//  k_decide     — gain ratio, damping update and commit of accepted poses.
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

// init: NULL, or per window (mu0, nu0, rejects0, skip); a skipped window
// starts stopped (done = 3), so no pass touches it.
__global__ void k_lm_reset(int32_t W, LMState *__restrict__ lm, double mu0, double nu0, int32_t rejects0,
                           const double *__restrict__ init, const int32_t *__restrict__ win_group_ptr) {
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= W) return;
    LMState s;
    s.mu = init ? init[4 * w] : mu0;
    s.nu = init ? init[4 * w + 1] : nu0;
    s.cost = 0.0; s.cost_trial = 0.0; s.q = 0.0; s.rho = 0.0;
    s.gnorm = 0.0; s.maxdiag = 0.0; s.cost0 = 0.0;
    s.accepted = 0; s.need_eval = 1; s.info = 0;
    s.done = (win_group_ptr[w + 1] == win_group_ptr[w]) ? 1 : 0;   // a window without voxels has nothing to do
    if (init && init[4 * w + 3] != 0.0) s.done = 3;
    s.iters = 0; s.n_accepted = 0; s.cur = 0;
    s.rejects = init ? (int32_t)init[4 * w + 2] : rejects0;
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

// The increment solve of windows of up to SPLIT_SOLVE_POSES poses: blocks of
// WSOLVE_BLOCK threads, blockIdx.y selecting a range of WSOLVE_BLOCK poses of
// window blockIdx.x.  When the derivatives are fresh every block forms the
// window's gradient norm and largest Hessian diagonal itself (all blocks
// compute the same bits; the window's first block records them) and applies
// the convergence test; then each block solves its poses' damped 6x6 systems
// and forms the trial poses T (+) dx.  Wider windows take two launches, the
// statistics in one block (k_window_stats_mm), then one thread per pose over
// the whole grid (k_solve_mm_lm).  The statistics always follow one order,
// that of a WSTAT_THREADS-thread pass: virtual thread v sums poses p0 + v,
// p0 + v + WSTAT_THREADS, ... (g_k^2 by fma in k order, max over the
// diagonal), and the virtual wave totals are added in wave order.  So the
// results do not depend on which form runs.
static constexpr int WSTAT_THREADS = 512;
static constexpr int WSOLVE_BLOCK = 256;
static constexpr int SPLIT_SOLVE_POSES = 1024;

// Window statistics in the WSTAT_THREADS order by a block of B threads, thread
// t playing virtual threads t, t + B, ...; `red` holds 2 * WSTAT_THREADS / 64
// doubles.  The block synchronises once; every thread returns the totals.
template <int B>
__device__ __forceinline__ void window_stats_ordered(const double *__restrict__ g, const double *__restrict__ H,
                                                     int p0, int p1, double *red, double &gs_out,
                                                     double &mx_out) {
    static_assert(WSTAT_THREADS % B == 0 && B % 64 == 0, "block must tile the statistics pass");
    constexpr int V = WSTAT_THREADS / B, NWB = B / 64, NW = WSTAT_THREADS / 64;
    double gs[V], mx[V];
#pragma unroll
    for (int v = 0; v < V; v++) gs[v] = mx[v] = 0.0;
    for (int base = p0 + threadIdx.x; base < p1; base += WSTAT_THREADS) {
#pragma unroll
        for (int v = 0; v < V; v++) {
            const int j = base + v * B;
            if (j < p1) {
#pragma unroll
                for (int k = 0; k < 6; k++) {
                    const double gk = g[6LL * j + k];
                    gs[v] = fma(gk, gk, gs[v]);
                    mx[v] = fmax(mx[v], H[36LL * j + 7 * k]);
                }
            }
        }
    }
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < V; v++) {
        gs[v] = wave_sum(gs[v]);
        mx[v] = wave_max(mx[v]);
    }
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int v = 0; v < V; v++) {
            red[v * NWB + wave] = gs[v];
            red[NW + v * NWB + wave] = mx[v];
        }
    }
    __syncthreads();
    double a = 0.0, m = red[NW];
#pragma unroll
    for (int i = 0; i < NW; i++) a += red[i];
#pragma unroll
    for (int i = 1; i < NW; i++) m = fmax(m, red[NW + i]);
    gs_out = a;
    mx_out = m;
}

// Records fresh statistics and the convergence test; returns whether the
// window has converged.
__device__ __forceinline__ bool record_stats(LMState &st, double gs, double mx, double tol_g, bool write) {
    const double gn = sqrt(gs);
    const bool conv = tol_g > 0.0 && gn < tol_g;
    if (write) {
        st.gnorm = gn;
        st.maxdiag = mx;
        if (conv) {
            st.done = 1;
            st.accepted = 0;
        }
    }
    return conv;
}

__global__ __launch_bounds__(WSOLVE_BLOCK) void k_window_solve_mm(
    int32_t W, const int32_t *__restrict__ win_pose_ptr, LMState *__restrict__ lm, const double *__restrict__ g,
    const double *__restrict__ H, const double *__restrict__ poses, double *__restrict__ dx,
    double *__restrict__ pose_q, int32_t *__restrict__ pose_info, double *__restrict__ poses_trial, double tol_g) {
    __shared__ double red[2 * (WSTAT_THREADS / 64)];
    __shared__ int s_done;
    const int w = blockIdx.x;
    if (w >= W) return;
    LMState &st = lm[w];
    // Only the window's first block writes st here, and only the statistics
    // (read by the other blocks only when the derivatives are not fresh) and
    // the converged flag (which every block derives itself as well).  The
    // flag is read once per block, so the block decides as one.
    // The state and index reads are issued together, before the barrier.
    const int p0 = win_pose_ptr[w], p1 = win_pose_ptr[w + 1];
    const int fresh = st.need_eval;
    const double mu = st.mu, md = fresh ? 0.0 : st.maxdiag;   // maxdiag is rewritten only when fresh
    if (threadIdx.x == 0) s_done = st.done;
    __syncthreads();
    if (s_done) return;
    const int j = p0 + (int)blockIdx.y * WSOLVE_BLOCK + (int)threadIdx.x;
    if (blockIdx.y > 0 && p0 + (int)blockIdx.y * WSOLVE_BLOCK >= p1) return;   // block-uniform
    double fl;
    if (fresh) {
        double gs, mx;
        window_stats_ordered<WSOLVE_BLOCK>(g, H, p0, p1, red, gs, mx);
        if (record_stats(st, gs, mx, tol_g, blockIdx.y == 0 && threadIdx.x == 0)) return;
        fl = 1e-12 * mx;
    } else {
        fl = 1e-12 * md;
    }
    if (j >= p1) return;
    double q;
    const int info = solve_pose(H + 36LL * j, g + 6LL * j, mu, fl, dx + 6LL * j, q);
    pose_q[j] = q;
    pose_info[j] = info ? 6 * (j - p0) + info : 0;
    pose_plus(poses + 12LL * j, dx + 6LL * j, poses_trial + 12LL * j);
}

__global__ __launch_bounds__(WSTAT_THREADS) void k_window_stats_mm(int32_t W,
                                                                   const int32_t *__restrict__ win_pose_ptr,
                                                                   LMState *__restrict__ lm,
                                                                   const double *__restrict__ g,
                                                                   const double *__restrict__ H, double tol_g) {
    __shared__ double red[2 * (WSTAT_THREADS / 64)];
    const int w = blockIdx.x;
    if (w >= W) return;
    LMState &st = lm[w];
    if (st.done || !st.need_eval) return;
    double gs, mx;
    window_stats_ordered<WSTAT_THREADS>(g, H, win_pose_ptr[w], win_pose_ptr[w + 1], red, gs, mx);
    (void)record_stats(st, gs, mx, tol_g, threadIdx.x == 0);
}

void launch_window_solve_mm(Problem *P, const double *poses, double tol_g, hipStream_t s) {
    int32_t widest = 0;
    for (int32_t w = 0; w < P->n_windows; w++)
        widest = std::max(widest, P->h_win_pose_ptr[w + 1] - P->h_win_pose_ptr[w]);
    ProfScope prof("k_window_solve_mm", s);
    if (widest > SPLIT_SOLVE_POSES) {
        hipLaunchKernelGGL(k_window_stats_mm, dim3(P->n_windows), dim3(WSTAT_THREADS), 0, s, P->n_windows,
                           P->win_pose_ptr, P->lm, P->g, P->H, tol_g);
        hipLaunchKernelGGL(k_solve_mm_lm, dim3((unsigned)((P->n_poses + 255) / 256)), dim3(256), 0, s, P->n_poses,
                           P->pose_window, P->win_pose_ptr, P->lm, P->H, P->g, poses, P->dx, P->pose_q, P->pose_info,
                           P->poses_trial);
        return;
    }
    const unsigned nb = (unsigned)std::max(1, (widest + WSOLVE_BLOCK - 1) / WSOLVE_BLOCK);
    hipLaunchKernelGGL(k_window_solve_mm, dim3(P->n_windows, nb), dim3(WSOLVE_BLOCK), 0, s, P->n_windows,
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

void launch_lm_reset(Problem *P, double mu0, double nu0, int32_t rejects0, const double *init, hipStream_t s) {
    hipLaunchKernelGGL(k_lm_reset, dim3(nblk(P->n_windows)), dim3(256), 0, s, P->n_windows, P->lm, mu0, nu0, rejects0,
                       init,
                       P->win_group_ptr);
}

void launch_lm_cost(Problem *P, hipStream_t s) {
    hipLaunchKernelGGL(k_lm_cost, dim3(P->n_windows), dim3(DECIDE_THREADS), 0, s, P->n_windows, P->win_group_ptr,
                       P->wave_cost, P->lm);
}

// Statistics and convergence test at the end of an MM run, in the order of
// the in-loop test (window_stats_ordered), so the reported gradient norm and
// flag are bitwise the ones the next iteration's solve would form.
void launch_window_stats(Problem *P, double tol_g, hipStream_t s) {
    hipLaunchKernelGGL(k_window_stats_mm, dim3(P->n_windows), dim3(WSTAT_THREADS), 0, s, P->n_windows,
                       P->win_pose_ptr, P->lm, P->g, P->H, tol_g);
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
