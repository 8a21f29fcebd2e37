// Evaluation kernels of one iteration (paper Alg. 2, CalRes and CalJH).
//
//  k_vox   — residual pass, one lane per voxel, one block per group of 64
//            voxels with equal cluster count (their clusters split over the
//            block's four waves).  Each lane transforms its voxel's clusters by
//            the current poses (Eq. 2), forms the voxel covariance A_i (Eq. 1)
//            by the parallel-axis theorem about a per-voxel reference point,
//            takes the smallest eigenpair with register-resident Jacobi
//            rotations, and stores (u, mbar, 2/N_i, lambda_min) for the
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

#include "ba.h"
#include "ba_device.hpp"
#include "ba_internal.hpp"
#include "ba_kernels.hpp"

namespace ba {

// Accumulates the clusters k = k0, k0 + kstep, ... of the voxel in `lane` of
// group g relative to the centroid r of the voxel's first cluster (which keeps
// the sums well conditioned at large coordinates):
//   n = sum N_k,  s = sum N_k d_k,  M = sum [St_k + N_k d_k d_k^T],  d_k = m_k - r.
struct VoxSums {
    double n, s0, s1, s2;
    double M[6];
    double r[3];
};

__device__ __forceinline__ void vox_accumulate(const GroupDesc &g, int lane, int k0, int kstep, int64_t c_pad,
                                               const double *__restrict__ vN, const double *__restrict__ vmu,
                                               const double *__restrict__ vS, const int32_t *__restrict__ vpose,
                                               const double *__restrict__ poses, VoxSums &a) {
    a.n = a.s0 = a.s1 = a.s2 = 0.0;
#pragma unroll
    for (int q = 0; q < 6; q++) a.M[q] = 0.0;
    {
        const int64_t idx = g.cbase + lane;
        const double mu[3] = {vmu[idx], vmu[c_pad + idx], vmu[2 * c_pad + idx]};
        Pose P;
        load_pose(poses, vpose[idx], P);
        rot(P.r, mu, a.r);
        a.r[0] += P.t[0]; a.r[1] += P.t[1]; a.r[2] += P.t[2];
    }
#pragma unroll 2
    for (int k = k0; k < g.m; k += kstep) {
        const int64_t idx = g.cbase + 64LL * k + lane;
        const double nk = vN[idx];
        const double mu[3] = {vmu[idx], vmu[c_pad + idx], vmu[2 * c_pad + idx]};
        double S[6];
#pragma unroll
        for (int q = 0; q < 6; q++) S[q] = vS[q * c_pad + idx];
        Pose P;
        load_pose(poses, vpose[idx], P);
        double y[3], St[6];
        rot(P.r, mu, y);
        rot_sym(P.r, S, St);
        const double d0 = (y[0] + P.t[0]) - a.r[0], d1 = (y[1] + P.t[1]) - a.r[1], d2 = (y[2] + P.t[2]) - a.r[2];
        const double nd0 = nk * d0, nd1 = nk * d1, nd2 = nk * d2;
        a.n += nk;
        a.s0 += nd0; a.s1 += nd1; a.s2 += nd2;
        a.M[0] += fma(nd0, d0, St[0]);
        a.M[1] += fma(nd0, d1, St[1]);
        a.M[2] += fma(nd0, d2, St[2]);
        a.M[3] += fma(nd1, d1, St[3]);
        a.M[4] += fma(nd1, d2, St[4]);
        a.M[5] += fma(nd2, d2, St[5]);
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
    double lam[3], u[3];
    eig_sym3(A, lam, u);
    st[0] = u[0]; st[1] = u[1]; st[2] = u[2];
    st[3] = a.r[0] + b0; st[4] = a.r[1] + b1; st[5] = a.r[2] + b2;
    st[6] = 2.0 * inv;
    st[7] = lam[0];
    return lam[0];
}

// Residual pass.  One block per group of 64 voxels with equal cluster count
// (blocks ordered largest count first); the four waves split the group's
// clusters (k = w, w + 4, ...) and wave 0 adds the partial sums in wave order.
// (The LM decision runs as its own kernel: a last-block-done ticket would need
// a device-scope fence per block, which writes back the XCD-private L2.)
__global__ __launch_bounds__(256) void k_vox(const VoxBlock *__restrict__ blocks, const GroupDesc *__restrict__ groups,
                                             int64_t c_pad, const double *__restrict__ vN,
                                             const double *__restrict__ vmu, const double *__restrict__ vS,
                                             const int32_t *__restrict__ vpose, const double *__restrict__ poses,
                                             double *__restrict__ vstate, int64_t n_slots,
                                             const LMState *__restrict__ lm, int trial,
                                             double *__restrict__ group_cost) {
    __shared__ double part[3][10][64];
    const VoxBlock b = blocks[blockIdx.x];
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    int buf = 0;
    if (lm) {
        const LMState &st = lm[b.window];
        if (st.done) return;
        buf = trial ? 1 - st.cur : st.cur;
    }
    double *vs = vstate + (int64_t)buf * n_slots * VSTATE;
    const int gi = b.g0;
    const GroupDesc g = groups[gi];
    const bool active = lane < g.nvox;
    VoxSums a;
    a.n = a.s0 = a.s1 = a.s2 = 0.0;
    for (int q = 0; q < 6; q++) a.M[q] = 0.0;
    if (active && w < g.m) vox_accumulate(g, lane, w, 4, c_pad, vN, vmu, vS, vpose, poses, a);
    if (w > 0) {
        double *pp = &part[w - 1][0][0];
        pp[lane] = a.n;
        pp[64 + lane] = a.s0; pp[128 + lane] = a.s1; pp[192 + lane] = a.s2;
#pragma unroll
        for (int q = 0; q < 6; q++) pp[(4 + q) * 64 + lane] = a.M[q];
    }
    __syncthreads();
    if (w == 0) {
        double lam0 = 0.0;
        if (active) {
            for (int v = 0; v < 3; v++) {
                const double *pp = &part[v][0][0];
                a.n += pp[lane];
                a.s0 += pp[64 + lane]; a.s1 += pp[128 + lane]; a.s2 += pp[192 + lane];
#pragma unroll
                for (int q = 0; q < 6; q++) a.M[q] += pp[(4 + q) * 64 + lane];
            }
            lam0 = vox_finish(a, vs + ((int64_t)gi * 64 + lane) * VSTATE);
        }
        const double c = wave_sum(lam0);
        if (lane == 0) group_cost[gi] = c;
    }
}

__global__ __launch_bounds__(256) void k_pose(const ChunkDesc *__restrict__ chunks, int32_t n_chunks, int64_t C,
                                              const double *__restrict__ pN, const double *__restrict__ pmu,
                                              const double *__restrict__ pS, const int32_t *__restrict__ pslot,
                                              const double *__restrict__ poses, const double *__restrict__ vstate,
                                              int64_t n_slots, const int32_t *__restrict__ pose_window,
                                              const LMState *__restrict__ lm, double *__restrict__ partials) {
    const int wave = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (wave >= n_chunks) return;
    const ChunkDesc ch = chunks[wave];
    int buf = 0;
    if (lm) {
        const LMState &st = lm[pose_window[ch.pose]];
        if (st.done || !st.need_eval) return;
        buf = st.cur;
    }
    Pose P;
    load_pose(poses, ch.pose, P);
    const double *vs = vstate + (int64_t)buf * n_slots * VSTATE;
    double acc[NPART];
#pragma unroll
    for (int q = 0; q < NPART; q++) acc[q] = 0.0;
    for (int i = lane; i < ch.count; i += 64) {
        const int64_t q = ch.start + i;
        const double n = pN[q];
        const double mu[3] = {pmu[q], pmu[C + q], pmu[2 * C + q]};
        double S[6];
#pragma unroll
        for (int k = 0; k < 6; k++) S[k] = pS[k * C + q];
        const double *st = vs + (int64_t)pslot[q] * VSTATE;
        const double u[3] = {st[0], st[1], st[2]};
        const double mb[3] = {st[3], st[4], st[5]};
        const double sc = st[6];
        double y[3], St[6];
        rot(P.r, mu, y);
        rot_sym(P.r, S, St);
        const double d[3] = {y[0] + P.t[0] - mb[0], y[1] + P.t[1] - mb[1], y[2] + P.t[2] - mb[2]};
        const double e = dot(u, d);
        double su[3];
        sym_mv(St, u, su);
        const double ne = n * e;
        const double w[3] = {fma(ne, y[0], su[0]), fma(ne, y[1], su[1]), fma(ne, y[2], su[2])};
        double wxu[3], a[3];
        cross(w, u, wxu);
        cross(y, u, a);
        // gradient
        acc[0] = fma(sc, wxu[0], acc[0]);
        acc[1] = fma(sc, wxu[1], acc[1]);
        acc[2] = fma(sc, wxu[2], acc[2]);
        const double sne = sc * ne;
        acc[3] = fma(sne, u[0], acc[3]);
        acc[4] = fma(sne, u[1], acc[4]);
        acc[5] = fma(sne, u[2], acc[5]);
        // [u]x St [u]x^T : B = [u]x St, C = B [u]x^T
        const double Sf[3][3] = {{St[0], St[1], St[2]}, {St[1], St[3], St[4]}, {St[2], St[4], St[5]}};
        const double K[3][3] = {{0.0, -u[2], u[1]}, {u[2], 0.0, -u[0]}, {-u[1], u[0], 0.0}};
        double B[3][3];
#pragma unroll
        for (int r = 0; r < 3; r++)
#pragma unroll
            for (int c = 0; c < 3; c++) B[r][c] = K[r][0] * Sf[0][c] + K[r][1] * Sf[1][c] + K[r][2] * Sf[2][c];
        double Cu[6];
        Cu[0] = B[0][0] * K[0][0] + B[0][1] * K[0][1] + B[0][2] * K[0][2];
        Cu[1] = B[0][0] * K[1][0] + B[0][1] * K[1][1] + B[0][2] * K[1][2];
        Cu[2] = B[0][0] * K[2][0] + B[0][1] * K[2][1] + B[0][2] * K[2][2];
        Cu[3] = B[1][0] * K[1][0] + B[1][1] * K[1][1] + B[1][2] * K[1][2];
        Cu[4] = B[1][0] * K[2][0] + B[1][1] * K[2][1] + B[1][2] * K[2][2];
        Cu[5] = B[2][0] * K[2][0] + B[2][1] * K[2][1] + B[2][2] * K[2][2];
        const double uw = dot(u, w);
        const int ii[6] = {0, 0, 0, 1, 1, 2}, jj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
        for (int k = 0; k < 6; k++) {
            const int r = ii[k], c = jj[k];
            double h = n * a[r] * a[c] + Cu[k] + 0.5 * (u[r] * w[c] + w[r] * u[c]);
            if (r == c) h -= uw;
            acc[6 + k] = fma(sc, h, acc[6 + k]);
        }
        const double sn = sc * n;
#pragma unroll
        for (int r = 0; r < 3; r++)
#pragma unroll
            for (int c = 0; c < 3; c++) acc[12 + 3 * r + c] = fma(sn * a[r], u[c], acc[12 + 3 * r + c]);
#pragma unroll
        for (int k = 0; k < 6; k++) acc[21 + k] = fma(sn * u[ii[k]], u[jj[k]], acc[21 + k]);
    }
    // reduce-scatter over the wave: lane l ends with the sum of value l / 2
    double red[32];
#pragma unroll
    for (int q = 0; q < 32; q++) red[q] = (q < NPART) ? acc[q] : 0.0;
    const double v = wave_reduce_scatter32(red, lane);
    if ((lane & 1) == 0 && (lane >> 1) < NPART) partials[(int64_t)wave * NPART + (lane >> 1)] = v;
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

// One block per window: fixed-order sum of the window's wave residuals.
__global__ __launch_bounds__(256) void k_window_cost(int32_t n_windows, const int32_t *__restrict__ win_group_ptr,
                                                     const double *__restrict__ wave_cost, double *__restrict__ out) {
    __shared__ double red[256];
    const int w = blockIdx.x;
    if (w >= n_windows) return;
    double s = 0.0;
    for (int i = win_group_ptr[w] + threadIdx.x; i < win_group_ptr[w + 1]; i += 256) s += wave_cost[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[w] = red[0];
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

void launch_vox(Problem *P, const double *poses, bool use_lm, bool trial, hipStream_t s) {
    if (P->n_vblocks == 0) return;
    ProfScope prof("k_vox", s);
    hipLaunchKernelGGL(k_vox, dim3((unsigned)P->n_vblocks), dim3(256), 0, s, P->vblocks, P->groups, P->c_pad, P->v_N,
                       P->v_mu, P->v_S, P->v_pose, poses, P->vstate, (int64_t)P->n_groups * 64,
                       use_lm ? P->lm : nullptr, trial ? 1 : 0, P->wave_cost);
}

void launch_window_cost(Problem *P, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_window_cost, dim3(P->n_windows), dim3(256), 0, s, P->n_windows, P->win_group_ptr,
                       P->wave_cost, out);
}

void launch_pose_chunks(Problem *P, const double *poses, bool use_lm, hipStream_t s) {
    if (P->n_chunks > 0) {
        ProfScope prof("k_pose", s);
        hipLaunchKernelGGL(k_pose, dim3(nblk((int64_t)P->n_chunks * 64)), dim3(256), 0, s, P->chunks, P->n_chunks,
                           P->n_clusters, P->p_N, P->p_mu, P->p_S, P->p_slot, poses, P->vstate,
                           (int64_t)P->n_groups * 64, P->pose_window, use_lm ? P->lm : nullptr, P->partials);
    }
}

void launch_pose_derivs(Problem *P, const double *poses, bool use_lm, double *g, double *H, hipStream_t s) {
    if (P->n_chunks > 0) {
        ProfScope prof("k_pose", s);
        hipLaunchKernelGGL(k_pose, dim3(nblk((int64_t)P->n_chunks * 64)), dim3(256), 0, s, P->chunks, P->n_chunks,
                           P->n_clusters, P->p_N, P->p_mu, P->p_S, P->p_slot, poses, P->vstate,
                           (int64_t)P->n_groups * 64, P->pose_window, use_lm ? P->lm : nullptr, P->partials);
    }
    hipLaunchKernelGGL(k_reduce_partials, dim3(nblk((int64_t)P->n_poses * NPART)), dim3(256), 0, s, P->n_poses,
                       P->chunk_ptr, P->partials, P->pose_window, use_lm ? P->lm : nullptr, g, H);
}

void launch_voxel_eig(Problem *P, double *out, hipStream_t s) {
    const int64_t ns = (int64_t)P->n_groups * 64;
    if (ns == 0) return;
    hipLaunchKernelGGL(k_voxel_eig, dim3(nblk(ns)), dim3(256), 0, s, ns, P->slot_vox, P->vstate, out);
}

}  // namespace ba
