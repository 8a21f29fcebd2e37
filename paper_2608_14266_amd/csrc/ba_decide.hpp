// Per-window Levenberg-Marquardt decision (reading of the unprinted
// PredResReduction / Adjust of Alg. 2): gain ratio, damping update, commit of
// accepted poses.  Executed by one 1024-thread block per window.
#pragma once
#include <hip/hip_runtime.h>

#include "ba_internal.hpp"

namespace ba {

static constexpr int DECIDE_THREADS = 1024;

// Sum of a window's group residuals [g0, g1) by a DECIDE_THREADS block, in
// one fixed order (used for the current, the trial and the reported cost):
// each thread's groups g0 + t, g0 + t + DECIDE_THREADS, ... in turn, then the
// block reduction in wave order.
__device__ __forceinline__ double window_cost_part(int g0, int g1, const double *__restrict__ group_cost) {
    double c = 0.0;
#pragma unroll 4
    for (int i = g0 + threadIdx.x; i < g1; i += DECIDE_THREADS) c += group_cost[i];
    return c;
}

__device__ __forceinline__ double window_cost_sum(int g0, int g1, const double *__restrict__ group_cost,
                                                  double *red) {
    return block_sum<DECIDE_THREADS / 64>(window_cost_part(g0, g1, group_cost), red);
}

// Copy of a window's 12 * n pose values, eight loads in flight per thread
// before their stores (the two arrays never overlap).
__device__ __forceinline__ void copy_window_poses(const double *__restrict__ src, double *__restrict__ dst,
                                                  int64_t n) {
    constexpr int U = 8;
    for (int64_t b = threadIdx.x; b < n; b += (int64_t)U * DECIDE_THREADS) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t i = b + (int64_t)u * DECIDE_THREADS;
            v[u] = i < n ? src[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t i = b + (int64_t)u * DECIDE_THREADS;
            if (i < n) dst[i] = v[u];
        }
    }
}

__device__ __forceinline__ void decide_window(int w, const DecideArgs &da) {
    constexpr int NW = DECIDE_THREADS / 64;
    __shared__ double red_q[NW], red_c[NW];
    __shared__ int redi[NW];
    __shared__ int s_acc;
    LMState &st = da.lm[w];
    if (st.done) return;
    double q = 0.0, c;
    int info = 0x7fffffff;
    const int p0 = da.win_pose_ptr[w], p1 = da.win_pose_ptr[w + 1];
    const int g0 = da.win_group_ptr[w], g1 = da.win_group_ptr[w + 1];
    for (int j = p0 + threadIdx.x; j < p1; j += DECIDE_THREADS) {
        q += da.pose_q[j];
        const int inf = da.pose_info[j];
        if (inf) info = min(info, inf);
    }
    c = window_cost_part(g0, g1, da.group_cost);
    block_sum2_min<NW>(q, c, info, red_q, red_c, redi);
    if (threadIdx.x == 0) {
        const double qq = q, ct = c;
        const int inf = (info == 0x7fffffff) ? 0 : info;
        const double rho = (inf == 0 && qq > 0.0) ? (st.cost - ct) / qq : -1.0;
        const int acc = rho > 0.0;
        if (da.trace) {
            double *t = da.trace + ((int64_t)da.it * da.W + w) * 8;
            t[0] = st.cost; t[1] = inf ? st.cost : ct; t[2] = rho; t[3] = st.mu;
            t[4] = acc; t[5] = st.gnorm; t[6] = inf; t[7] = inf ? 0.0 : qq;
        }
        s_acc = acc;
        st.q = qq;
        st.rho = rho;
        st.info = inf;
        st.cost_trial = ct;
        st.accepted = acc;
        st.iters += 1;
        if (acc) {
            st.cost = ct;
            st.cur = 1 - st.cur;
            st.need_eval = 1;
            st.n_accepted += 1;
            const double f = 2.0 * rho - 1.0;
            const double fac = 1.0 - f * f * f;
            st.mu *= (fac > 1.0 / 3.0 ? fac : 1.0 / 3.0);
            st.nu = 2.0;
            st.rejects = 0;
        } else {
            st.need_eval = 0;
            st.mu *= st.nu;
            st.nu *= 2.0;
            st.rejects += 1;
            if (da.max_rejects > 0 && st.rejects >= da.max_rejects) st.done = 2;
        }
    }
    __syncthreads();
    if (s_acc) copy_window_poses(da.poses_trial + 12LL * p0, da.poses + 12LL * p0, 12LL * (p1 - p0));
}

}  // namespace ba
