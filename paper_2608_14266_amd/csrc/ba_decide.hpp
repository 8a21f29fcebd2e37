// Per-window Levenberg-Marquardt decision (reading of the unprinted
// PredResReduction / Adjust of Alg. 2): gain ratio, damping update, commit of
// accepted poses.  Executed by one 256-thread block per window.
#pragma once
#include <hip/hip_runtime.h>

#include "ba_internal.hpp"

namespace ba {

__device__ __forceinline__ void decide_window(int w, const DecideArgs &da) {
    __shared__ double rq[256], rc[256];
    __shared__ int ri[256];
    __shared__ int s_acc;
    LMState &st = da.lm[w];
    if (st.done) return;
    double q = 0.0, c = 0.0;
    int info = 0x7fffffff;
    const int p0 = da.win_pose_ptr[w], p1 = da.win_pose_ptr[w + 1];
    const int g0 = da.win_group_ptr[w], g1 = da.win_group_ptr[w + 1];
#pragma unroll 4
    for (int j = p0 + threadIdx.x; j < p1; j += 256) {
        q += da.pose_q[j];
        const int inf = da.pose_info[j];
        if (inf) info = min(info, inf);
    }
#pragma unroll 8
    for (int i = g0 + threadIdx.x; i < g1; i += 256) c += da.group_cost[i];
    rq[threadIdx.x] = q;
    rc[threadIdx.x] = c;
    ri[threadIdx.x] = info;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            rq[threadIdx.x] += rq[threadIdx.x + o];
            rc[threadIdx.x] += rc[threadIdx.x + o];
            ri[threadIdx.x] = min(ri[threadIdx.x], ri[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double qq = rq[0], ct = rc[0];
        const int inf = (ri[0] == 0x7fffffff) ? 0 : ri[0];
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
        } else {
            st.mu *= st.nu;
            st.nu *= 2.0;
        }
    }
    __syncthreads();
    if (s_acc) {
        const int64_t a = 12LL * p0, b = 12LL * p1;
#pragma unroll 4
        for (int64_t i = a + threadIdx.x; i < b; i += 256) da.poses[i] = da.poses_trial[i];
    }
}

}  // namespace ba
