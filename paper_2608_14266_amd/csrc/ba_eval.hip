// Evaluation kernels of one iteration (paper Alg. 2, CalRes and CalJH).
//
//  k_vox   — residual pass, one lane per voxel, one block per group of 64
//            voxels with equal cluster count (their clusters split over the
//            block's four waves).  Each lane transforms its voxel's clusters by
//            the current poses (Eq. 2), forms the voxel covariance A_i (Eq. 1)
//            by the parallel-axis theorem about a per-voxel reference point,
//            takes the smallest eigenpair in registers (Newton shift on the
//            characteristic polynomial, then Rayleigh quotient iteration on
//            the adjugate), and stores (u, mbar, 2/N_i, lambda_min) for the
//            derivative pass.  The residual of a group is reduced in-wave.
//  k_pose  — derivative pass, one wavefront per pose chunk (clusters of one
//            scan, pose-major copy).  Each lane evaluates the per-cluster
//            gradient and Hessian of the Eq. 3 surrogate from its cluster and
//            its voxel's frozen (u, mbar) and accumulates them in registers;
//            the wave reduces the 27 sums once per chunk.  This is the
//            reduce_by_key over poses of Alg. 2 without the scatter M_s and
//            without floating-point atomics.
//  k_reduce_partials — sums each pose's chunk partials in a fixed order and
//            expands g (6) and H (6x6) per pose.
//
// Per cluster (voxel i, scan j), with ybar = R mu, m = ybar + t, St = R S R^T,
// e = u^T (m - mbar), w = N_ij e ybar + St u, a = ybar x u and s = 2 / N_i:
//   g_ij = s [ w x u ; N_ij e u ]
//   H_ij = s [[ N_ij a a^T + [u]x St [u]x^T + (u w^T + w u^T)/2 - (u^T w) I , N_ij a u^T ],
//             [ N_ij u a^T , N_ij u u^T ]]
// (the Hessian of Eq. 3 in the chart (Exp(phi) R, t + dt); the paper defers
// these derivatives to BALM3, they are derived from Eq. 3 directly).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ba.h"
#include "ba_device.hpp"
#include "ba_internal.hpp"
#include "ba_kernels.hpp"
#include "ba_decide.hpp"

namespace ba {

// Accumulates the clusters k = k0, k0 + kstep, ... of the voxel in `lane` of
// group g relative to a reference point r of the voxel (which keeps the sums
// well conditioned at large coordinates):
//   n = sum N_k,  s = sum N_k d_k,  M = sum [St_k + N_k d_k d_k^T],  d_k = m_k - r.
struct VoxSums {
    double n, s0, s1, s2;
    double M[6];
    double r[3];
};

// Cluster sources of the two precisions.  FP64: (N, mu, S) as built.  FP32
// (precision form): (N, mu', S') with mu' = R0 mu + t0 - c_i and
// S' = R0 S R0^T, in the world frame of the scan's reference pose T0 and
// relative to the voxel's reference point c_i (`ref`, per slot).
struct SrcF64 {
    const double *N, *mu, *S;
};
struct SrcF32 {
    const float *N, *mu, *S;
    const double *ref_poses;   // [n_poses][12]
    const double *ref;         // [slots][4]
    const double *pdelta;      // [n_poses][16] pose changes of the evaluated poses: E (9), w (3) (residual pass)
    const int32_t *cidx;       // [C] (voxel, scan)-order index of each pose-major cluster
    double *h;                 // [C][6] coupled pair vectors, written when not null
};

// Pose change of every scan for the precision form's residual pass:
// E = R R0^T - I and w = dt - E t0 with dt = t - t0 (one thread per pose),
// so that a cluster's offset from its voxel's reference point c is
// d = mu' + E (mu' + c) + w.
__global__ void k_pose_delta(int32_t n, const double *__restrict__ poses, const double *__restrict__ ref_poses,
                             double *__restrict__ pdelta) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    Pose P, P0;
    load_pose(poses, j, P);
    load_pose(ref_poses, j, P0);
    PoseDelta D;
    pose_delta(P, P0, D);
    double Et0[3];
    rot(D.E, P0.t, Et0);
    double *o = pdelta + 16LL * j;
#pragma unroll
    for (int e = 0; e < 9; e++) o[e] = D.E[e];
#pragma unroll
    for (int e = 0; e < 3; e++) o[9 + e] = D.dt[e] - Et0[e];
#pragma unroll
    for (int e = 12; e < 16; e++) o[e] = 0.0;
}

template <typename T>
__device__ __forceinline__ void vox_add(VoxSums &a, T nk, const T *d, const T *St) {
    const T nd0 = nk * d[0], nd1 = nk * d[1], nd2 = nk * d[2];
    a.n += (double)nk;
    a.s0 += (double)nd0; a.s1 += (double)nd1; a.s2 += (double)nd2;
    a.M[0] += (double)fmaT(nd0, d[0], St[0]);
    a.M[1] += (double)fmaT(nd0, d[1], St[1]);
    a.M[2] += (double)fmaT(nd0, d[2], St[2]);
    a.M[3] += (double)fmaT(nd1, d[1], St[3]);
    a.M[4] += (double)fmaT(nd1, d[2], St[4]);
    a.M[5] += (double)fmaT(nd2, d[2], St[5]);
}

__device__ __forceinline__ void vox_zero(VoxSums &a) {
    a.n = a.s0 = a.s1 = a.s2 = 0.0;
#pragma unroll
    for (int q = 0; q < 6; q++) a.M[q] = 0.0;
}

// The per-scan operands a cluster gathers in the residual pass, 12 doubles
// per scan: the pose (R, t; FP64 clusters) or the pose change (E, w; FP32
// clusters).  A wave group's clusters observe a short run of scans (the
// voxels are ordered by their first observing scan), so a block copies the
// run into LDS once and its lanes gather from there instead of from the
// cache, when the group spans at most VOX_STAGE scans.
static constexpr int VOX_STAGE = 32;
static constexpr int VOX_ROW = 12;

__device__ __forceinline__ const double *vox_table(const SrcF64 &, const double *poses, int &stride) {
    stride = 12;
    return poses;
}
__device__ __forceinline__ const double *vox_table(const SrcF32 &src, const double *, int &stride) {
    stride = 16;
    return src.pdelta;
}

// All threads of the block: the scan rows of groups g0 .. g0 + ng - 1 into
// rows[q * VOX_STAGE * VOX_ROW ..] (groups that span more scans are skipped).
// The caller synchronises before the rows are read.
template <class Src>
__device__ __forceinline__ void vox_stage(const GroupDesc *__restrict__ groups, int g0, int ng, const Src &src,
                                          const double *__restrict__ poses, double *__restrict__ rows) {
    int stride;
    const double *tab = vox_table(src, poses, stride);
    for (int e = threadIdx.x; e < ng * VOX_STAGE * VOX_ROW; e += blockDim.x) {
        const int q = e / (VOX_STAGE * VOX_ROW), r = e % (VOX_STAGE * VOX_ROW);
        const int s = r / VOX_ROW, k = r % VOX_ROW;
        const GroupDesc g = groups[g0 + q];
        if (g.nscan <= VOX_STAGE && s < g.nscan) rows[e] = tab[(int64_t)(g.scan0 + s) * stride + k];
    }
}

// FP64: the reference is the centroid of the lane's first cluster.  srow:
// the group's staged scan rows in LDS, or null (gathers from `poses`).
__device__ __forceinline__ void vox_accumulate(const GroupDesc &g, int64_t slot, int lane, int k0, int kstep,
                                               int64_t c_pad, const SrcF64 &src, const int32_t *__restrict__ vpose,
                                               const double *__restrict__ poses, const double *__restrict__ srow,
                                               VoxSums &a) {
    vox_zero(a);
    {
        const int64_t idx = g.cbase + lane;
        const double mu[3] = {src.mu[idx], src.mu[c_pad + idx], src.mu[2 * c_pad + idx]};
        Pose P;
        load_pose(poses, vpose[idx], P);
        rot(P.r, mu, a.r);
        a.r[0] += P.t[0]; a.r[1] += P.t[1]; a.r[2] += P.t[2];
    }
    // the scan id of the next cluster is loaded one iteration ahead, so the
    // pose gather does not wait for a dependent round trip
    int j_next = (k0 < g.m) ? vpose[g.cbase + 64LL * k0 + lane] : 0;
#pragma unroll 2
    for (int k = k0; k < g.m; k += kstep) {
        const int64_t idx = g.cbase + 64LL * k + lane;
        const int j = j_next;
        if (k + kstep < g.m) j_next = vpose[idx + 64LL * kstep];
        const double nk = src.N[idx];
        const double mu[3] = {src.mu[idx], src.mu[c_pad + idx], src.mu[2 * c_pad + idx]};
        double S[6];
#pragma unroll
        for (int q = 0; q < 6; q++) S[q] = src.S[q * c_pad + idx];
        Pose P;
        if (srow) {
            const double *q = srow + VOX_ROW * (j - g.scan0);
#pragma unroll
            for (int e = 0; e < 9; e++) P.r[e] = q[e];
#pragma unroll
            for (int e = 0; e < 3; e++) P.t[e] = q[9 + e];
        } else {
            load_pose(poses, j, P);
        }
        double y[3], St[6];
        rot(P.r, mu, y);
        rot_sym(P.r, S, St);
        const double d[3] = {(y[0] + P.t[0]) - a.r[0], (y[1] + P.t[1]) - a.r[1], (y[2] + P.t[2]) - a.r[2]};
        vox_add(a, nk, d, St);
    }
}

// FP32 storage: the reference is the voxel's reference point c.  With the
// pose change (E, w) of the cluster's scan, d = m - c = mu' + E (mu' + c) + w
// (w = dt - E t0: the reference translation is folded in per scan, so each
// cluster gathers 12 doubles of its scan, not 15), and St = S' + D(E, S').
// The arithmetic stays FP64: the residual feeds the LM gain ratio, whose cost
// differences reach 1e-12 relative near convergence, below the noise of any
// FP32 product here; E c and E t0 round at about 1e-16 |E| |c|.
__device__ __forceinline__ void vox_accumulate(const GroupDesc &g, int64_t slot, int lane, int k0, int kstep,
                                               int64_t c_pad, const SrcF32 &src, const int32_t *__restrict__ vpose,
                                               const double *__restrict__ poses, const double *__restrict__ srow,
                                               VoxSums &a) {
    vox_zero(a);
    const double *c = src.ref + 4 * slot;
    a.r[0] = c[0]; a.r[1] = c[1]; a.r[2] = c[2];
    int j_next = (k0 < g.m) ? vpose[g.cbase + 64LL * k0 + lane] : 0;
#pragma unroll 1
    for (int k = k0; k < g.m; k += kstep) {
        const int64_t idx = g.cbase + 64LL * k + lane;
        const int j = j_next;
        if (k + kstep < g.m) j_next = vpose[idx + 64LL * kstep];
        const double nk = (double)src.N[idx];
        const double mu[3] = {(double)src.mu[idx], (double)src.mu[c_pad + idx], (double)src.mu[2 * c_pad + idx]};
        double S[6];
#pragma unroll
        for (int q = 0; q < 6; q++) S[q] = (double)src.S[q * c_pad + idx];
        // pose change of scan j, formed once per evaluation (k_pose_delta)
        double E[9], w[3];
        if (srow) {
            const double *pd = srow + VOX_ROW * (j - g.scan0);
#pragma unroll
            for (int e = 0; e < 9; e++) E[e] = pd[e];
#pragma unroll
            for (int e = 0; e < 3; e++) w[e] = pd[9 + e];
        } else {
            const double *pd = src.pdelta + 16LL * j;
#pragma unroll
            for (int e = 0; e < 9; e++) E[e] = pd[e];
#pragma unroll
            for (int e = 0; e < 3; e++) w[e] = pd[9 + e];
        }
        const double mc[3] = {mu[0] + a.r[0], mu[1] + a.r[1], mu[2] + a.r[2]};
        double Emc[3], Dl[6];
        rot(E, mc, Emc);
        delta_sym(E, S, Dl);
        const double d[3] = {mu[0] + (Emc[0] + w[0]), mu[1] + (Emc[1] + w[1]), mu[2] + (Emc[2] + w[2])};
        double St[6];
#pragma unroll
        for (int e = 0; e < 6; e++) St[e] = S[e] + Dl[e];
        vox_add(a, nk, d, St);
    }
}

// mbar = r + s / n,  A = (M - s s^T / n) / n;  smallest eigenpair; voxel state.
__device__ __forceinline__ double vox_finish(const VoxSums &a, double *__restrict__ st) {
    const double inv = 1.0 / a.n;
    const double b0 = a.s0 * inv, b1 = a.s1 * inv, b2 = a.s2 * inv;
    double A[6];
    A[0] = (a.M[0] - a.s0 * b0) * inv;
    A[1] = (a.M[1] - a.s0 * b1) * inv;
    A[2] = (a.M[2] - a.s0 * b2) * inv;
    A[3] = (a.M[3] - a.s1 * b1) * inv;
    A[4] = (a.M[4] - a.s1 * b2) * inv;
    A[5] = (a.M[5] - a.s2 * b2) * inv;
    double lam0, u[3];
    eig_min_sym3_safe(A, lam0, u);
    st[0] = u[0]; st[1] = u[1]; st[2] = u[2];
    st[3] = a.r[0] + b0; st[4] = a.r[1] + b1; st[5] = a.r[2] + b2;
    st[6] = 2.0 * inv;
    st[7] = lam0;
    return lam0;
}

// Stores the records of a group's nvox voxels (64 bytes each, contiguous in
// LDS at R) to their slots: every store instruction of the block covers whole
// consecutive lines, where each lane storing its own record would touch 64
// lines with 16 bytes each.
__device__ __forceinline__ void store_records(const double *R, double *__restrict__ dst, int nvox) {
    const double2 *src = reinterpret_cast<const double2 *>(R);
    double2 *d = reinterpret_cast<double2 *>(dst);
    for (int p = threadIdx.x; p < 4 * nvox; p += blockDim.x) d[p] = src[p];
}

template <class Src, int SPLIT>
__device__ __forceinline__ void vox_item(int bi, const VoxBlock *__restrict__ blocks,
                                         const GroupDesc *__restrict__ groups, int64_t c_pad, const Src &src,
                                         const int32_t *__restrict__ vpose, const double *__restrict__ poses,
                                         double *__restrict__ vstate, int64_t n_slots,
                                         const LMState *__restrict__ lm, int trial,
                                         double *__restrict__ group_cost, double (*part)[10][64],
                                         double *__restrict__ rows) {
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const VoxBlock b = blocks[bi];
    int buf = 0;
    if (lm) {
        const LMState &st = lm[b.window];
        if (st.done) return;       // uniform over the block
        buf = trial ? 1 - st.cur : st.cur;
    }
    double *vs = vstate + (int64_t)buf * n_slots * VSTATE;
    const int gi = b.g0;
    const GroupDesc g = groups[gi];
    vox_stage(groups, gi, 1, src, poses, rows);
    __syncthreads();
    const double *srow = g.nscan <= VOX_STAGE ? rows : nullptr;
    const bool active = lane < g.nvox;
    VoxSums a;
    vox_zero(a);
    if (active && w < g.m)
        vox_accumulate(g, (int64_t)gi * 64 + lane, lane, w, SPLIT, c_pad, src, vpose, poses, srow, a);
    if (SPLIT > 1 && w > 0) {
        double *pp = &part[w - 1][0][0];
        pp[lane] = a.n;
        pp[64 + lane] = a.s0; pp[128 + lane] = a.s1; pp[192 + lane] = a.s2;
#pragma unroll
        for (int q = 0; q < 6; q++) pp[(4 + q) * 64 + lane] = a.M[q];
    }
    if (SPLIT > 1) __syncthreads();
    if (w == 0) {
        double lam0 = 0.0;
        double rec[VSTATE];
        if (active) {
            for (int v = 0; v < SPLIT - 1; v++) {
                const double *pp = &part[v][0][0];
                a.n += pp[lane];
                a.s0 += pp[64 + lane]; a.s1 += pp[128 + lane]; a.s2 += pp[192 + lane];
#pragma unroll
                for (int q = 0; q < 6; q++) a.M[q] += pp[(4 + q) * 64 + lane];
            }
            lam0 = vox_finish(a, rec);
            // the group's records through LDS (part[0], read above by this wave only)
            double *R = &part[0][0][0];
#pragma unroll
            for (int k = 0; k < VSTATE; k++) R[lane * VSTATE + k] = rec[k];
        }
        const double c = wave_sum(lam0);
        if (lane == 0) group_cost[gi] = c;
    }
    __syncthreads();
    store_records(&part[0][0][0], vs + (int64_t)gi * 64 * VSTATE, g.nvox);
}

// Residual pass.  One work item per group of 64 voxels with equal cluster
// count (items ordered largest count first); the block's SPLIT waves share
// the group's clusters (k = w, w + SPLIT, ...) and wave 0 adds the partial
// sums in wave order.  With a persistent grid (PERSIST) each block walks the
// item list with a stride of the grid size.  (The LM decision runs as its own
// kernel: a last-block-done ticket would need a device-scope fence per block,
// which writes back the XCD-private L2.)
template <class Src, int SPLIT, bool PERSIST>
__global__ __launch_bounds__(64 * SPLIT) void k_vox(const VoxBlock *__restrict__ blocks, int32_t n_blocks,
                                                    const GroupDesc *__restrict__ groups, int64_t c_pad, Src src,
                                                    const int32_t *__restrict__ vpose,
                                                    const double *__restrict__ poses, double *__restrict__ vstate,
                                                    int64_t n_slots, const LMState *__restrict__ lm, int trial,
                                                    double *__restrict__ group_cost) {
    __shared__ double part[SPLIT > 1 ? SPLIT - 1 : 1][10][64];
    __shared__ double rows[VOX_STAGE * VOX_ROW];
    if constexpr (!PERSIST) {
        vox_item<Src, SPLIT>((int)blockIdx.x, blocks, groups, c_pad, src, vpose, poses, vstate, n_slots, lm, trial,
                             group_cost, part, rows);
    } else {
        for (int bi = blockIdx.x; bi < n_blocks; bi += gridDim.x) {
            vox_item<Src, SPLIT>(bi, blocks, groups, c_pad, src, vpose, poses, vstate, n_slots, lm, trial,
                                 group_cost, part, rows);
            __syncthreads();   // part[] and rows[] are reused by the next item
        }
    }
}

// Residual pass with the split chosen per group (plan table vblocks_mix):
// a 256-thread block takes 4 / split groups of one window, `split` waves per
// group sharing its clusters (k = part, part + split, ...); the first wave of
// each group adds the others' partial sums in wave order through LDS and
// finishes the voxels.  Every wave reaches the one barrier.
template <class Src, bool PERSIST>
__global__ __launch_bounds__(256) void k_vox_mixed(const VoxBlock *__restrict__ blocks, int32_t n_blocks,
                                                   const GroupDesc *__restrict__ groups, int64_t c_pad, Src src,
                                                   const int32_t *__restrict__ vpose,
                                                   const double *__restrict__ poses, double *__restrict__ vstate,
                                                   int64_t n_slots, const LMState *__restrict__ lm, int trial,
                                                   double *__restrict__ group_cost) {
    __shared__ double part[4][10][64];
    __shared__ double rows[4][VOX_STAGE * VOX_ROW];
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    for (int bi = blockIdx.x; bi < n_blocks; bi += (PERSIST ? gridDim.x : n_blocks)) {
        const VoxBlock b = blocks[bi];
        const int sp = b.split;
        const int gsub = w / sp, pt = w % sp;
        const bool has_group = gsub < b.ng;
        const int gi = b.g0 + (has_group ? gsub : 0);
        vox_stage(groups, b.g0, b.ng, src, poses, &rows[0][0]);
        __syncthreads();
        int buf = 0;
        bool run = has_group;
        if (lm) {
            const LMState &st = lm[b.window];
            run = run && !st.done;
            buf = trial ? 1 - st.cur : st.cur;
        }
        const GroupDesc g = groups[gi];
        const double *srow = g.nscan <= VOX_STAGE ? rows[gsub] : nullptr;
        const bool active = run && lane < g.nvox;
        VoxSums a;
        vox_zero(a);
        if (active && pt < g.m)
            vox_accumulate(g, (int64_t)gi * 64 + lane, lane, pt, sp, c_pad, src, vpose, poses, srow, a);
        if (pt > 0) {
            double *pp = &part[w][0][0];
            pp[lane] = a.n;
            pp[64 + lane] = a.s0; pp[128 + lane] = a.s1; pp[192 + lane] = a.s2;
#pragma unroll
            for (int q = 0; q < 6; q++) pp[(4 + q) * 64 + lane] = a.M[q];
        }
        __syncthreads();
        if (pt == 0 && run) {
            double lam0 = 0.0;
            double rec[VSTATE];
            if (active) {
                for (int v = 1; v < sp; v++) {
                    const double *pp = &part[w + v][0][0];
                    a.n += pp[lane];
                    a.s0 += pp[64 + lane]; a.s1 += pp[128 + lane]; a.s2 += pp[192 + lane];
#pragma unroll
                    for (int q = 0; q < 6; q++) a.M[q] += pp[(4 + q) * 64 + lane];
                }
                lam0 = vox_finish(a, rec);
                // the group's records through this wave's own (unused) part[w]
                double *R = &part[w][0][0];
#pragma unroll
                for (int k = 0; k < VSTATE; k++) R[lane * VSTATE + k] = rec[k];
            }
            const double c = wave_sum(lam0);
            if (lane == 0) group_cost[gi] = c;
        }
        __syncthreads();
        if (pt == 0 && run) {
            // the finishing wave stores its group's records as whole lines
            const double2 *src2 = reinterpret_cast<const double2 *>(&part[w][0][0]);
            double2 *d = reinterpret_cast<double2 *>(vstate + ((int64_t)buf * n_slots + (int64_t)gi * 64) * VSTATE);
            for (int p = lane; p < 4 * g.nvox; p += 64) d[p] = src2[p];
        }
        if (PERSIST) __syncthreads();   // part[] is reused by the next item
    }
}

// Per-cluster surrogate gradient and Hessian terms (formulas in the header of
// this file) in arithmetic T from y = R mu (lever arm), e = u^T (m - mbar)
// (FP64), St and u, with the voxel scale sc = 2 / N_i: the gradient terms
// added into FP64 accumulators (acc), the 21 Hessian terms into accumulators
// of type H (hacc).
template <typename T, typename H>
__device__ __forceinline__ void pose_terms(T n, const T *y, double e64, const T *St, const T *u, double sc,
                                           double *acc, H *hacc, bool grad = true) {
    const T e = (T)e64;
    T su[3];
    sym_mv(St, u, su);
    const T ne = n * e;
    const T w[3] = {fmaT(ne, y[0], su[0]), fmaT(ne, y[1], su[1]), fmaT(ne, y[2], su[2])};
    T a[3];
    cross(y, u, a);
    if (grad) {
        T wxu[3];
        cross(w, u, wxu);
        acc[0] = fma(sc, (double)wxu[0], acc[0]);
        acc[1] = fma(sc, (double)wxu[1], acc[1]);
        acc[2] = fma(sc, (double)wxu[2], acc[2]);
        const double sne = sc * ((double)n * e64);
        acc[3] = fma(sne, (double)u[0], acc[3]);
        acc[4] = fma(sne, (double)u[1], acc[4]);
        acc[5] = fma(sne, (double)u[2], acc[5]);
    }
    // [u]x St [u]x^T for symmetric St, expanded: with u = (a, b, c) each entry
    // is a combination of the six products of u's components
    const T ua = u[0], ub = u[1], uc = u[2];
    const T aa = ua * ua, bb = ub * ub, cc = uc * uc, ab = ua * ub, ac = ua * uc, bc = ub * uc;
    T Cu[6];
    Cu[0] = cc * St[3] - T(2) * bc * St[4] + bb * St[5];
    Cu[1] = bc * St[2] - cc * St[1] + ac * St[4] - ab * St[5];
    Cu[2] = bc * St[1] - bb * St[2] - ac * St[3] + ab * St[4];
    Cu[3] = aa * St[5] - T(2) * ac * St[2] + cc * St[0];
    Cu[4] = ab * St[2] - bc * St[0] + ac * St[1] - aa * St[4];
    Cu[5] = bb * St[0] - T(2) * ab * St[1] + aa * St[3];
    const T uw = dot(u, w);
    const int ii[6] = {0, 0, 0, 1, 1, 2}, jj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int k = 0; k < 6; k++) {
        const int r = ii[k], c = jj[k];
        T h = n * a[r] * a[c] + Cu[k] + T(0.5) * (u[r] * w[c] + w[r] * u[c]);
        if (r == c) h -= uw;
        hacc[k] = fmaT((H)sc, (H)h, hacc[k]);
    }
    const H sn = (H)(sc * (double)n);
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
        for (int c = 0; c < 3; c++) hacc[6 + 3 * r + c] = fmaT(sn * (H)a[r], (H)u[c], hacc[6 + 3 * r + c]);
#pragma unroll
    for (int k = 0; k < 6; k++) hacc[15 + k] = fmaT(sn * (H)u[ii[k]], (H)u[jj[k]], hacc[15 + k]);
}

// Pose context of a chunk: the pose, and for the FP32 form its reference
// pose, the pose change (E, dt) and E rounded to FP32.
struct PoseCtx {
    Pose P, P0;
    PoseDelta D;
    float E[9];
};

__device__ __forceinline__ void pose_cluster(const SrcF64 &src, const PoseCtx &cx, int64_t q, int64_t C,
                                             const double *st, int32_t slot, double *acc) {
    const double n = src.N[q];
    const double mu[3] = {src.mu[q], src.mu[C + q], src.mu[2 * C + q]};
    double S[6];
#pragma unroll
    for (int k = 0; k < 6; k++) S[k] = src.S[k * C + q];
    const double u[3] = {st[0], st[1], st[2]};
    double y[3], St[6];
    rot(cx.P.r, mu, y);
    rot_sym(cx.P.r, S, St);
    const double d[3] = {y[0] + cx.P.t[0] - st[3], y[1] + cx.P.t[1] - st[4], y[2] + cx.P.t[2] - st[5]};
    pose_terms(n, y, dot(u, d), St, u, st[6], acc, acc + 6);
}

// FP32 form: with q = c - t0 and G = I + E the pose change,
//   y = R mu = G mu' + G q,   d = m - mbar = G mu' + (E q + dt + c - mbar);
// y, the plane offset e = u^T d and the gradient terms in FP64 from the FP32
// cluster; D(E, S') and the Hessian terms in FP32 (FP64 in the coupled form).
template <bool HESS64>
__device__ __forceinline__ void pose_cluster(const SrcF32 &src, const PoseCtx &cx, int64_t q, int64_t C,
                                             const double *st, int32_t slot, double *acc, float *hacc) {
    const float n = src.N[q];
    const double mu[3] = {(double)src.mu[q], (double)src.mu[C + q], (double)src.mu[2 * C + q]};
    float S[6];
#pragma unroll
    for (int k = 0; k < 6; k++) S[k] = src.S[k * C + q];
    const double *c = src.ref + 4LL * slot;
    const double qv[3] = {c[0] - cx.P0.t[0], c[1] - cx.P0.t[1], c[2] - cx.P0.t[2]};
    // FP64: G mu' = mu' + E mu', the lever arm y = G mu' + G q and the plane
    // offset e = u^T (G mu' + E q + dt + c - mbar)
    double Em[3], Eq[3], y64[3];
    rot(cx.D.E, mu, Em);
    rot(cx.D.E, qv, Eq);
    double e = 0.0;
#pragma unroll
    for (int i = 0; i < 3; i++) {
        const double gm = mu[i] + Em[i];
        y64[i] = gm + (qv[i] + Eq[i]);
        e = fma(st[i], gm + ((Eq[i] + cx.D.dt[i]) + (c[i] - st[3 + i])), e);
    }
    const double u64[3] = {st[0], st[1], st[2]};
    if constexpr (HESS64) {
        if (src.h) {
            // h = (N_ij / N_i) [y x u ; u] of the coupled form
            const double f = (double)n * (0.5 * st[6]);
            double a[3];
            cross(y64, u64, a);
            double *o = src.h + 6 * q;   // pose-major order (the pair plan indexes it so)
            o[0] = f * a[0]; o[1] = f * a[1]; o[2] = f * a[2];
            o[3] = f * u64[0]; o[4] = f * u64[1]; o[5] = f * u64[2];
        }
        double Sd[6], Dl64[6], S64[6];
#pragma unroll
        for (int k = 0; k < 6; k++) Sd[k] = (double)S[k];
        delta_sym(cx.D.E, Sd, Dl64);
#pragma unroll
        for (int k = 0; k < 6; k++) S64[k] = Sd[k] + Dl64[k];
        pose_terms((double)n, y64, e, S64, u64, st[6], acc, acc + 6);
        return;
    }
    // St = S' + D(E, S') with D in FP32 (of the size of the pose change)
    float Dl[6];
    delta_sym(cx.E, S, Dl);
    // gradient terms in FP64: the iteration converges to where they cancel,
    // so their rounding sets the accuracy of the result; the Hessian terms
    // (most of the arithmetic) only steer the steps and stay FP32, except for
    // the coupled form (HESS64), whose dense Newton-like step amplifies their
    // rounding along the nearly singular gauge directions; they are summed
    // per lane in FP32 (at most 16 terms between FP64 additions)
    {
        double S64[6], su[3];
#pragma unroll
        for (int k = 0; k < 6; k++) S64[k] = (double)S[k] + (double)Dl[k];
        sym_mv(S64, u64, su);
        const double ne = (double)n * e;
        const double w[3] = {fma(ne, y64[0], su[0]), fma(ne, y64[1], su[1]), fma(ne, y64[2], su[2])};
        double wxu[3];
        cross(w, u64, wxu);
        const double sc = st[6];
        acc[0] = fma(sc, wxu[0], acc[0]);
        acc[1] = fma(sc, wxu[1], acc[1]);
        acc[2] = fma(sc, wxu[2], acc[2]);
        const double sne = sc * ne;
        acc[3] = fma(sne, u64[0], acc[3]);
        acc[4] = fma(sne, u64[1], acc[4]);
        acc[5] = fma(sne, u64[2], acc[5]);
    }
    const float u[3] = {(float)st[0], (float)st[1], (float)st[2]};
    const float y[3] = {(float)y64[0], (float)y64[1], (float)y64[2]};
    float St[6];
#pragma unroll
    for (int k = 0; k < 6; k++) St[k] = S[k] + Dl[k];
    pose_terms(n, y, e, St, u, st[6], acc, hacc, false);
}

// Block b of a launch runs on XCD b mod 8.  Renumbering the blocks so that
// XCD x receives one contiguous range of the work list gives each XCD's L2
// the chunks of neighbouring poses, which observe the same voxels: their
// voxel-state lines are then fetched once per XCD instead of once per cluster.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    constexpr int X = 8;
    const int q = nb / X, r = nb % X;
    const int x = b % X, i = b / X;
    return x * q + min(x, r) + i;
}

// Derivative pass: one wavefront per pose chunk, blocks renumbered per XCD.
// With a persistent grid each wave walks the chunk list with a stride of the
// number of waves.
template <class Src, bool PERSIST, bool HESS64>
__global__ __launch_bounds__(256) void k_pose(const ChunkDesc *__restrict__ chunks, int32_t n_chunks, int64_t C,
                                              Src src, const int32_t *__restrict__ pslot,
                                              const double *__restrict__ poses, const double *__restrict__ vstate,
                                              int64_t n_slots, const int32_t *__restrict__ pose_window,
                                              const LMState *__restrict__ lm, double *__restrict__ partials) {
    const int lane = threadIdx.x & 63;
    const int n_waves = (int)((gridDim.x * blockDim.x) >> 6);
    const int blk = xcd_block((int)blockIdx.x, (int)gridDim.x);
    for (int wave = (int)(((int64_t)blk * blockDim.x + threadIdx.x) >> 6); wave < n_chunks;
         wave += (PERSIST ? n_waves : n_chunks)) {
        const ChunkDesc ch = chunks[wave];
        int buf = 0;
        if (lm) {
            const LMState &st = lm[pose_window[ch.pose]];
            if (st.done || !st.need_eval) continue;   // uniform over the wave
            buf = st.cur;
        }
        PoseCtx cx;
        load_pose(poses, ch.pose, cx.P);
        if constexpr (sizeof(*src.N) == 4) {
            load_pose(src.ref_poses, ch.pose, cx.P0);
            pose_delta(cx.P, cx.P0, cx.D);
#pragma unroll
            for (int k = 0; k < 9; k++) cx.E[k] = (float)cx.D.E[k];
        }
        const double *vs = vstate + (int64_t)buf * n_slots * VSTATE;
        double acc[NPART];
#pragma unroll
        for (int q = 0; q < NPART; q++) acc[q] = 0.0;
        // precision form: the FP32 Hessian terms summed per lane in FP32 (a
        // chunk holds at most MAX_CHUNK clusters: 16 terms per lane), then
        // converted once for the FP64 reduction
        float hacc[NPART - 6];
#pragma unroll
        for (int q = 0; q < NPART - 6; q++) hacc[q] = 0.0f;
#pragma unroll 1
        for (int i = lane; i < ch.count; i += 64) {
            const int64_t q = ch.start + i;
            const int32_t slot = pslot[q];
            if constexpr (sizeof(*src.N) == 4)
                pose_cluster<HESS64>(src, cx, q, C, vs + (int64_t)slot * VSTATE, slot, acc, hacc);
            else
                pose_cluster(src, cx, q, C, vs + (int64_t)slot * VSTATE, slot, acc);
        }
        if constexpr (sizeof(*src.N) == 4 && !HESS64) {
#pragma unroll
            for (int q = 0; q < NPART - 6; q++) acc[6 + q] = (double)hacc[q];
        }
        // reduce-scatter over the wave: lane l ends with the sum of value l / 2
        double red[32];
#pragma unroll
        for (int q = 0; q < 32; q++) red[q] = (q < NPART) ? acc[q] : 0.0;
        const double v = wave_reduce_scatter32(red, lane);
        if ((lane & 1) == 0 && (lane >> 1) < NPART) partials[(int64_t)wave * NPART + (lane >> 1)] = v;
    }
}

// One thread per (pose, component): fixed-order sum over the pose's chunks.
__global__ void k_reduce_partials(int32_t n_poses, const int32_t *__restrict__ chunk_ptr,
                                  const double *__restrict__ partials, const int32_t *__restrict__ pose_window,
                                  const LMState *__restrict__ lm, double *__restrict__ g, double *__restrict__ H) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (int64_t)n_poses * NPART) return;
    const int j = (int)(tid / NPART), k = (int)(tid % NPART);
    if (lm) {
        const LMState &st = lm[pose_window[j]];
        if (st.done || !st.need_eval) return;
    }
    double s = 0.0;
    const int c0 = chunk_ptr[j], c1 = chunk_ptr[j + 1];
#pragma unroll 4
    for (int c = c0; c < c1; c++) s += partials[(int64_t)c * NPART + k];
    double *h = H + 36LL * j;
    if (k < 6) {
        g[6LL * j + k] = s;
    } else if (k < 12) {
        const int ii[6] = {0, 0, 0, 1, 1, 2}, jj[6] = {0, 1, 2, 1, 2, 2};
        const int r = ii[k - 6], c = jj[k - 6];
        h[6 * r + c] = s;
        h[6 * c + r] = s;
    } else if (k < 21) {
        const int r = (k - 12) / 3, c = (k - 12) % 3;
        h[6 * r + 3 + c] = s;
        h[6 * (3 + c) + r] = s;
    } else {
        const int ii[6] = {0, 0, 0, 1, 1, 2}, jj[6] = {0, 1, 2, 1, 2, 2};
        const int r = 3 + ii[k - 21], c = 3 + jj[k - 21];
        h[6 * r + c] = s;
        h[6 * c + r] = s;
    }
}

// One block per window: the window's residual, summed in the order the LM
// decision uses.
__global__ __launch_bounds__(DECIDE_THREADS) void k_window_cost(int32_t n_windows,
                                                                const int32_t *__restrict__ win_group_ptr,
                                                                const double *__restrict__ wave_cost,
                                                                double *__restrict__ out) {
    __shared__ double red[DECIDE_THREADS / 64];
    const int w = blockIdx.x;
    if (w >= n_windows) return;
    const double c = window_cost_sum(win_group_ptr[w], win_group_ptr[w + 1], wave_cost, red);
    if (threadIdx.x == 0) out[w] = c;
}

// (lambda_min, u) per input voxel id
__global__ void k_voxel_eig(int64_t n_slots, const int32_t *__restrict__ slot_vox, const double *__restrict__ vstate,
                            double *__restrict__ out) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_slots) return;
    const int32_t v = slot_vox[s];
    if (v < 0) return;
    const double *st = vstate + s * VSTATE;
    out[4LL * v + 0] = st[7];
    out[4LL * v + 1] = st[0];
    out[4LL * v + 2] = st[1];
    out[4LL * v + 3] = st[2];
}

static inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

static SrcF64 src64(Problem *P, bool vox, bool = false) {
    return vox ? SrcF64{P->v_N, P->v_mu, P->v_S} : SrcF64{P->p_N, P->p_mu, P->p_S};
}
static SrcF32 src32(Problem *P, bool vox, bool hvec = false) {
    return vox ? SrcF32{P->v_N32, P->v_mu32, P->v_S32, P->ref_poses, P->v_ref, P->pdelta, nullptr, nullptr}
               : SrcF32{P->p_N32, P->p_mu32, P->p_S32, P->ref_poses, P->v_ref, nullptr, P->p_cidx,
                        hvec ? dense_hvec(P) : nullptr};
}

// Grid of a pass with `items` work items: one block per item, or a
// persistent grid of `per_cu` blocks per compute unit.
static unsigned pass_grid(int64_t items, int per_item_blocks_div, int per_cu, int n_cu) {
    const int64_t full = (items + per_item_blocks_div - 1) / per_item_blocks_div;
    if (per_cu <= 0) return (unsigned)std::max<int64_t>(full, 1);
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(full, (int64_t)per_cu * n_cu));
}

void launch_vox(Problem *P, const double *poses, bool use_lm, bool trial, hipStream_t s) {
    if (P->n_vblocks == 0) return;
    ProfScope prof("k_vox", s);
    const int64_t ns = (int64_t)P->n_groups * 64;
    const LMState *lm = use_lm ? P->lm : nullptr;
    const dim3 grid(pass_grid(P->n_vblocks, 1, P->tune.vox_grid, P->n_cu));
    const int t = trial ? 1 : 0;
    if (P->prec == BA_PREC_F32)
        hipLaunchKernelGGL(k_pose_delta, dim3(nblk(P->n_poses)), dim3(256), 0, s, P->n_poses, poses, P->ref_poses,
                           P->pdelta);
    const bool pers = P->tune.vox_grid > 0;
#define BA_VOX(SRC, SPL, MK)                                                                                       \
    do {                                                                                                           \
        if (pers)                                                                                                  \
            hipLaunchKernelGGL((k_vox<SRC, SPL, true>), grid, dim3(64 * SPL), 0, s, P->vblocks, P->n_vblocks,      \
                               P->groups, P->c_pad, MK(P, true), P->v_pose, poses, P->vstate, ns, lm, t,           \
                               P->wave_cost);                                                                      \
        else                                                                                                       \
            hipLaunchKernelGGL((k_vox<SRC, SPL, false>), grid, dim3(64 * SPL), 0, s, P->vblocks, P->n_vblocks,     \
                               P->groups, P->c_pad, MK(P, true), P->v_pose, poses, P->vstate, ns, lm, t,           \
                               P->wave_cost);                                                                      \
    } while (0)
#define BA_VOX_MIX(SRC, MK)                                                                                       \
    do {                                                                                                           \
        const dim3 gm(pass_grid(P->n_vblocks_mix, 1, P->tune.vox_grid, P->n_cu));                                   \
        if (pers)                                                                                                  \
            hipLaunchKernelGGL((k_vox_mixed<SRC, true>), gm, dim3(256), 0, s, P->vblocks_mix, P->n_vblocks_mix,    \
                               P->groups, P->c_pad, MK(P, true), P->v_pose, poses, P->vstate, ns, lm, t,           \
                               P->wave_cost);                                                                      \
        else                                                                                                       \
            hipLaunchKernelGGL((k_vox_mixed<SRC, false>), gm, dim3(256), 0, s, P->vblocks_mix, P->n_vblocks_mix,   \
                               P->groups, P->c_pad, MK(P, true), P->v_pose, poses, P->vstate, ns, lm, t,           \
                               P->wave_cost);                                                                      \
    } while (0)
    if (P->tune.vox_split == 0) {
        if (P->prec == BA_PREC_F32) BA_VOX_MIX(SrcF32, src32);
        else BA_VOX_MIX(SrcF64, src64);
    } else if (P->prec == BA_PREC_F32) {
        if (P->tune.vox_split == 1) BA_VOX(SrcF32, 1, src32);
        else if (P->tune.vox_split == 2) BA_VOX(SrcF32, 2, src32);
        else BA_VOX(SrcF32, 4, src32);
    } else {
        if (P->tune.vox_split == 1) BA_VOX(SrcF64, 1, src64);
        else if (P->tune.vox_split == 2) BA_VOX(SrcF64, 2, src64);
        else BA_VOX(SrcF64, 4, src64);
    }
#undef BA_VOX
}

void launch_window_cost(Problem *P, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_window_cost, dim3(P->n_windows), dim3(DECIDE_THREADS), 0, s, P->n_windows, P->win_group_ptr,
                       P->wave_cost, out);
}

void launch_pose_chunks(Problem *P, const double *poses, bool use_lm, hipStream_t s, bool hess64) {
    if (P->n_chunks == 0) return;
    ProfScope prof("k_pose", s);
    const int64_t ns = (int64_t)P->n_groups * 64;
    const LMState *lm = use_lm ? P->lm : nullptr;
    const dim3 grid(pass_grid(P->n_chunks, 4, P->tune.pose_grid, P->n_cu));
    const bool pers = P->tune.pose_grid > 0;
#define BA_POSE(SRC, PER, H64, MK)                                                                                 \
    hipLaunchKernelGGL((k_pose<SRC, PER, H64>), grid, dim3(256), 0, s, P->chunks, P->n_chunks, P->n_clusters,     \
                       MK(P, false, H64), P->p_slot, poses, P->vstate, ns, P->pose_window, lm, P->partials)
    if (P->prec == BA_PREC_F32) {
        if (hess64) {
            if (pers) BA_POSE(SrcF32, true, true, src32);
            else BA_POSE(SrcF32, false, true, src32);
        } else {
            if (pers) BA_POSE(SrcF32, true, false, src32);
            else BA_POSE(SrcF32, false, false, src32);
        }
    } else {
        if (pers) BA_POSE(SrcF64, true, false, src64);
        else BA_POSE(SrcF64, false, false, src64);
    }
#undef BA_POSE
}

void launch_pose_derivs(Problem *P, const double *poses, bool use_lm, double *g, double *H, hipStream_t s,
                        bool hess64) {
    launch_pose_chunks(P, poses, use_lm, s, hess64);
    hipLaunchKernelGGL(k_reduce_partials, dim3(nblk((int64_t)P->n_poses * NPART)), dim3(256), 0, s, P->n_poses,
                       P->chunk_ptr, P->partials, P->pose_window, use_lm ? P->lm : nullptr, g, H);
}

void launch_voxel_eig(Problem *P, double *out, hipStream_t s) {
    const int64_t ns = (int64_t)P->n_groups * 64;
    if (ns == 0) return;
    hipLaunchKernelGGL(k_voxel_eig, dim3(nblk(ns)), dim3(256), 0, s, ns, P->slot_vox, P->vstate, out);
}

}  // namespace ba

