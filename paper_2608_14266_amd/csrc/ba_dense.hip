// Coupled Hessian and its dense damped solve.
//
// The first-stage majorizer u^T A_i(T) u of Eq. 1 (u frozen at T_l) keeps the
// poses coupled: its Hessian is the block diagonal of the Eq. 3 surrogate
// minus 2 h_ij h_ik^T for every pair of scans (j, k) observing voxel i, with
//     h_ij = (N_ij / N_i) [ (R_j mu_ij) x u ; u ].
// Assembly is deterministic and atomic-free: the plan lists every (voxel,
// j <= k) contribution sorted by the pose-pair key (j, k); one wavefront sums
// each key's contributions in a fixed order and writes that 6x6 block (and
// its transpose) of the dense per-window matrix.
//
// The damped system (H + mu D) dx = -g is solved by a right-looking blocked
// Cholesky with 64-wide panels (Alg. 2's Solver replaced by a dense one in
// this coupled form): the diagonal block is factored and inverted in LDS,
// the panel solve (P L^-T) and the trailing update (C -= P_I P_J^T) run on
// FP64 matrix cores (v_mfma_f64_16x16x4f64), the forward substitution rides
// along the panel steps, and the backward substitution sweeps the block
// rows.  Every kernel is batched over independent windows (blockIdx.y).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "ba.h"
#include "ba_device.hpp"
#include "ba_internal.hpp"
#include "ba_kernels.hpp"

namespace ba {

typedef double d4 __attribute__((ext_vector_type(4)));

static constexpr int TB = 64;         // tile / panel width
static constexpr int LDK = 33;        // LDS row stride of a 32-wide K chunk (padded)

// One dense matrix of the batch.
struct DenseDesc {
    int64_t a_off;     // doubles: start of the n x n row-major matrix
    int64_t linv_off;  // doubles: start of ceil(n/64) inverted 64x64 diagonal blocks
    int64_t v_off;     // doubles: start of the n-vector (right-hand side / forward result)
    int32_t n;
    int32_t pose0;     // first scan of the window (LM use)
};

// Per-matrix solve parameters.
struct DenseParam {
    double mu;
    double floor_;
    int32_t active;
    int32_t info;
};

// ---------------------------------------------------------------- assembly
// h_c = (N_c / N_i) [ (R mu_c) x u ; u ] for every cluster (voxel-major order)
__global__ void k_hvec(int64_t C, const double *__restrict__ cN, const double *__restrict__ cmu,
                       const int32_t *__restrict__ cscan, const int32_t *__restrict__ cslot,
                       const double *__restrict__ poses, const double *__restrict__ vstate, int64_t n_slots,
                       const int32_t *__restrict__ pose_window, const LMState *__restrict__ lm,
                       double *__restrict__ h) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    const int j = cscan[c];
    int buf = 0;
    if (lm) {
        const LMState &st = lm[pose_window[j]];
        if (st.done || !st.need_eval) return;
        buf = st.cur;
    }
    const double *st = vstate + ((int64_t)buf * n_slots + cslot[c]) * VSTATE;
    const double u[3] = {st[0], st[1], st[2]};
    const double f = cN[c] * (0.5 * st[6]);
    Pose P;
    load_pose(poses, j, P);
    const double mu[3] = {cmu[3 * c], cmu[3 * c + 1], cmu[3 * c + 2]};
    double y[3], a[3];
    rot(P.r, mu, y);
    cross(y, u, a);
    double *o = h + 6 * c;
    o[0] = f * a[0]; o[1] = f * a[1]; o[2] = f * a[2];
    o[3] = f * u[0]; o[4] = f * u[1]; o[5] = f * u[2];
}

__global__ void k_fill(int64_t n, double *__restrict__ p, double v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

struct PairSeg {
    int64_t start;
    int32_t count;
    int32_t ja, jb;   // scans, ja <= jb
    int32_t pad;
};

// One wavefront per pose-pair key: block(ja, jb) = [H_MM(ja) if ja == jb] - 2 sum h_a h_b^T
__global__ __launch_bounds__(256) void k_pairs(int32_t n_seg, const PairSeg *__restrict__ segs,
                                               const int32_t *__restrict__ pa, const int32_t *__restrict__ pb,
                                               const double *__restrict__ h, const double *__restrict__ Hmm,
                                               const int32_t *__restrict__ pose_window,
                                               const int32_t *__restrict__ win_pose_ptr,
                                               const int64_t *__restrict__ win_off, const LMState *__restrict__ lm,
                                               double *__restrict__ dense) {
    const int wave = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (wave >= n_seg) return;
    const PairSeg sg = segs[wave];
    const int w = pose_window[sg.ja];
    if (lm) {
        const LMState &st = lm[w];
        if (st.done || !st.need_eval) return;
    }
    double acc[64];
#pragma unroll
    for (int q = 0; q < 64; q++) acc[q] = 0.0;
    for (int i = lane; i < sg.count; i += 64) {
        const int64_t a = pa[sg.start + i], b = pb[sg.start + i];
        double ha[6], hb[6];
#pragma unroll
        for (int q = 0; q < 6; q++) {
            ha[q] = h[6 * a + q];
            hb[q] = h[6 * b + q];
        }
#pragma unroll
        for (int r = 0; r < 6; r++)
#pragma unroll
            for (int s = 0; s < 6; s++) acc[6 * r + s] = fma(ha[r], hb[s], acc[6 * r + s]);
    }
    // lane l < 36 ends with the wave total of entry l of the 6x6 block
    const double v = wave_reduce_scatter64(acc, lane);
    if (lane < 36) {
        const int r = lane / 6, s = lane % 6;
        const int p0 = win_pose_ptr[w];
        const int64_t nw = 6LL * (win_pose_ptr[w + 1] - p0);
        const int la = sg.ja - p0, lb = sg.jb - p0;
        double *D = dense + win_off[w];
        double out = -2.0 * v;
        if (sg.ja == sg.jb) out += Hmm[36LL * sg.ja + 6 * r + s];
        D[(6LL * la + r) * nw + 6 * lb + s] = out;
        if (sg.ja != sg.jb) D[(6LL * lb + s) * nw + 6 * la + r] = out;
    }
}

// ---------------------------------------------------------------- exact Hessian (diagnostic)
// The exact Hessian of Eq. 1 adds, per voxel, sum_l 2 / (l0 - l_l) F^l F^l^T
// (l = 1, 2) to the coupled one, with per cluster
//     F^l_c = (1/N_i) [ w0 x u_l + w_l x u0 ; N_c (e0 u_l + e_l u0) ],
//     w_k = N_c e_k ybar + St u_k,  e_k = u_k^T (m_c - mbar),
// (ybar = R mu_c, m_c = ybar + t, St = R S_c R^T).  All pair terms are
// negative semi-definite outer products, so each cluster carries three scaled
// vectors v_0 = sqrt(2) h, v_l = sqrt(2 / (l_l - l0)) F^l and a pair block is
// -sum_k v_k,a v_k,b^T.  Terms of a gap l_l - l0 <= 1e-12 l2 are dropped.
// One thread per voxel recomputes the voxel covariance at the poses and its
// full eigen-decomposition from the centred clusters (voxel-major order).
__global__ void k_exact_vecs(int32_t n_vx, const int64_t *__restrict__ vptr, const double *__restrict__ cN,
                             const double *__restrict__ cmu, const double *__restrict__ cS,
                             const int32_t *__restrict__ cscan, const double *__restrict__ poses,
                             double *__restrict__ ev) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n_vx) return;
    const int64_t a = vptr[v], b = vptr[v + 1];
    double Nv = 0.0, mb[3] = {0, 0, 0};
    for (int64_t c = a; c < b; c++) {
        Pose P;
        load_pose(poses, cscan[c], P);
        const double n = cN[c];
        double y[3];
        rot(P.r, cmu + 3 * c, y);
#pragma unroll
        for (int r = 0; r < 3; r++) mb[r] += n * (y[r] + P.t[r]);
        Nv += n;
    }
#pragma unroll
    for (int r = 0; r < 3; r++) mb[r] /= Nv;
    double A[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t c = a; c < b; c++) {
        Pose P;
        load_pose(poses, cscan[c], P);
        const double n = cN[c];
        double y[3], St[6], d[3];
        rot(P.r, cmu + 3 * c, y);
        rot_sym(P.r, cS + 6 * c, St);
#pragma unroll
        for (int r = 0; r < 3; r++) d[r] = y[r] + P.t[r] - mb[r];
        A[0] += St[0] + n * d[0] * d[0];
        A[1] += St[1] + n * d[0] * d[1];
        A[2] += St[2] + n * d[0] * d[2];
        A[3] += St[3] + n * d[1] * d[1];
        A[4] += St[4] + n * d[1] * d[2];
        A[5] += St[5] + n * d[2] * d[2];
    }
#pragma unroll
    for (int k = 0; k < 6; k++) A[k] /= Nv;
    double lam[3], U[9];
    eig_sym3_full(A, lam, U);
    const double tol = 1e-12 * fabs(lam[2]);
    double wl[3] = {sqrt(2.0), 0.0, 0.0};
    for (int l = 1; l <= 2; l++) {
        const double gap = lam[l] - lam[0];
        wl[l] = gap > tol ? sqrt(2.0 / gap) : 0.0;
    }
    const double *u0 = U;
    for (int64_t c = a; c < b; c++) {
        Pose P;
        load_pose(poses, cscan[c], P);
        const double n = cN[c];
        double y[3], St[6], d[3], w0[3], su[3], ya[3];
        rot(P.r, cmu + 3 * c, y);
        rot_sym(P.r, cS + 6 * c, St);
#pragma unroll
        for (int r = 0; r < 3; r++) d[r] = y[r] + P.t[r] - mb[r];
        const double e0 = dot(u0, d);
        sym_mv(St, u0, su);
#pragma unroll
        for (int r = 0; r < 3; r++) w0[r] = n * e0 * y[r] + su[r];
        double *o = ev + 18 * c;
        cross(y, u0, ya);
#pragma unroll
        for (int r = 0; r < 3; r++) {
            o[r] = wl[0] * (n / Nv) * ya[r];
            o[3 + r] = wl[0] * (n / Nv) * u0[r];
        }
        for (int l = 1; l <= 2; l++) {
            const double *ul = U + 3 * l;
            const double el = dot(ul, d);
            double sl[3], wlv[3], x1[3], x2[3];
            sym_mv(St, ul, sl);
#pragma unroll
            for (int r = 0; r < 3; r++) wlv[r] = n * el * y[r] + sl[r];
            cross(w0, ul, x1);
            cross(wlv, u0, x2);
#pragma unroll
            for (int r = 0; r < 3; r++) {
                o[6 * l + r] = wl[l] * (x1[r] + x2[r]) / Nv;
                o[6 * l + 3 + r] = wl[l] * n * (e0 * ul[r] + el * u0[r]) / Nv;
            }
        }
    }
}

// One wavefront per pose-pair key: block(ja, jb) = [H_MM(ja) if ja == jb]
// - sum over the key's cluster pairs of sum_k v_k,a v_k,b^T, with k over the
// coupled vector only for windows that take the coupled form (exact_below:
// the exact terms are used while the window's gradient norm is below it; a
// null lm uses them everywhere).
__global__ __launch_bounds__(256) void k_pairs_x(int32_t n_seg, const PairSeg *__restrict__ segs,
                                                 const int32_t *__restrict__ pa, const int32_t *__restrict__ pb,
                                                 const double *__restrict__ ev, const double *__restrict__ Hmm,
                                                 const int32_t *__restrict__ pose_window,
                                                 const int32_t *__restrict__ win_pose_ptr,
                                                 const int64_t *__restrict__ win_off, const LMState *__restrict__ lm,
                                                 double exact_below, double *__restrict__ dense) {
    const int wave = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (wave >= n_seg) return;
    const PairSeg sg = segs[wave];
    const int w = pose_window[sg.ja];
    int nk = 3;
    if (lm) {
        const LMState &st = lm[w];
        if (st.done || !st.need_eval) return;
        if (!(st.gnorm < exact_below)) nk = 1;
    }
    double acc[64];
#pragma unroll
    for (int q = 0; q < 64; q++) acc[q] = 0.0;
    for (int i = lane; i < sg.count; i += 64) {
        const int64_t a = pa[sg.start + i], b = pb[sg.start + i];
        for (int k = 0; k < nk; k++) {
            double va[6], vb[6];
#pragma unroll
            for (int q = 0; q < 6; q++) {
                va[q] = ev[18 * a + 6 * k + q];
                vb[q] = ev[18 * b + 6 * k + q];
            }
#pragma unroll
            for (int r = 0; r < 6; r++)
#pragma unroll
                for (int t = 0; t < 6; t++) acc[6 * r + t] = fma(va[r], vb[t], acc[6 * r + t]);
        }
    }
    const double v = wave_reduce_scatter64(acc, lane);
    if (lane < 36) {
        const int r = lane / 6, t = lane % 6;
        const int p0 = win_pose_ptr[w];
        const int64_t nw = 6LL * (win_pose_ptr[w + 1] - p0);
        const int la = sg.ja - p0, lb = sg.jb - p0;
        double *D = dense + win_off[w];
        double out = -v;
        if (sg.ja == sg.jb) out += Hmm[36LL * sg.ja + 6 * r + t];
        D[(6LL * la + r) * nw + 6 * lb + t] = out;
        if (sg.ja != sg.jb) D[(6LL * lb + t) * nw + 6 * la + r] = out;
    }
}

// ---------------------------------------------------------------- MFMA tile helpers
// acc += A_chunk (64x32) * B_chunk (64x32)^T for this wave's 32x32 quadrant.
// v_mfma_f64_16x16x4f64 operand layout on gfx950 (lane l): A[l%16][l/16],
// B[l/16][l%16]; accumulator register r holds D[l/16 + 4r][l%16].
__device__ __forceinline__ void mma_chunk(const double *__restrict__ As, const double *__restrict__ Bs,
                                          d4 acc[2][2]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r0 = 32 * (w >> 1), c0 = 32 * (w & 1);
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int kk = 0; kk < 32; kk += 4) {
        const double a0 = As[(r0 + li) * LDK + kk + lk];
        const double a1 = As[(r0 + 16 + li) * LDK + kk + lk];
        const double b0 = Bs[(c0 + li) * LDK + kk + lk];
        const double b1 = Bs[(c0 + 16 + li) * LDK + kk + lk];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
}

// The 8 elements of a 64 x 32 chunk this thread stages (rows r0.., columns
// k0..k0+31 of a row-major matrix; zero outside rows < nr, columns < nc).
__device__ __forceinline__ void load_chunk(double (&v)[8], const double *__restrict__ M, int64_t ld, int64_t r0,
                                           int64_t k0, int64_t nr, int64_t nc) {
#pragma unroll
    for (int e = 0; e < 8; e++) {
        const int idx = threadIdx.x + 256 * e;
        const int row = idx >> 5, col = idx & 31;
        const int64_t gr = r0 + row, gc = k0 + col;
        v[e] = (gr < nr && gc < nc) ? M[gr * ld + gc] : 0.0;
    }
}

__device__ __forceinline__ void store_chunk(double *__restrict__ lds, const double (&v)[8]) {
#pragma unroll
    for (int e = 0; e < 8; e++) {
        const int idx = threadIdx.x + 256 * e;
        lds[(idx >> 5) * LDK + (idx & 31)] = v[e];
    }
}

// acc += A(rows ra.., cols ka..ka+kw-1) * B(rows rb.., cols kb..kb+kw-1)^T for
// a 64 x 64 tile (kw a multiple of 32).  The next K chunk is loaded into
// registers while the matrix cores work on the current one.
__device__ __forceinline__ void tile_gemm_nt_acc(double *__restrict__ As, double *__restrict__ Bs,
                                                 const double *__restrict__ A, int64_t lda, int64_t ra, int64_t ka,
                                                 int64_t nra, int64_t nca, const double *__restrict__ B, int64_t ldb,
                                                 int64_t rb, int64_t kb, int64_t nrb, int64_t ncb, d4 acc[2][2],
                                                 int kw) {
    double va[8], vb[8];
    load_chunk(va, A, lda, ra, ka, nra, nca);
    load_chunk(vb, B, ldb, rb, kb, nrb, ncb);
    for (int kc = 0; kc < kw; kc += 32) {
        store_chunk(As, va);
        store_chunk(Bs, vb);
        __syncthreads();
        if (kc + 32 < kw) {
            load_chunk(va, A, lda, ra, ka + kc + 32, nra, nca);
            load_chunk(vb, B, ldb, rb, kb + kc + 32, nrb, ncb);
        }
        mma_chunk(As, Bs, acc);
        __syncthreads();
    }
}

// The same product into a cleared accumulator.
__device__ __forceinline__ void tile_gemm_nt(double *__restrict__ As, double *__restrict__ Bs,
                                             const double *__restrict__ A, int64_t lda, int64_t ra, int64_t ka,
                                             int64_t nra, int64_t nca, const double *__restrict__ B, int64_t ldb,
                                             int64_t rb, int64_t kb, int64_t nrb, int64_t ncb, d4 acc[2][2],
                                             int kw = 64) {
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    tile_gemm_nt_acc(As, Bs, A, lda, ra, ka, nra, nca, B, ldb, rb, kb, nrb, ncb, acc, kw);
}

// element (row, col) of the 64x64 tile held in acc[rb][cb][r] by this lane
#define ACC_ROW(rb, r) (32 * ((threadIdx.x >> 6) >> 1) + 16 * (rb) + ((threadIdx.x & 63) >> 4) + 4 * (r))
#define ACC_COL(cb) (32 * ((threadIdx.x >> 6) & 1) + 16 * (cb) + (threadIdx.x & 15))

// ---------------------------------------------------------------- factorization
// A = H + mu max(diag H, floor) ; v = -g
__global__ void k_damp_copy(const DenseDesc *__restrict__ desc, const DenseParam *__restrict__ prm,
                            const double *__restrict__ H, const int64_t *__restrict__ h_off,
                            const double *__restrict__ g, double *__restrict__ work) {
    const int m = blockIdx.y;
    const DenseDesc d = desc[m];
    const DenseParam p = prm[m];
    if (!p.active) return;
    const int64_t nn = (int64_t)d.n * d.n;
    const double *Hm = H + h_off[m];
    double *A = work + d.a_off;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nn; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / d.n, c = i % d.n;
        double v = Hm[i];
        if (r == c) v += p.mu * (v > p.floor_ ? v : p.floor_);
        A[i] = v;
    }
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < d.n) work[d.v_off + t] = -g[6LL * d.pose0 + t];
}

// Broadcast lane `src` (wave-uniform) of a wave-wide double to every lane.
__device__ __forceinline__ double bcast(double v, int src) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

// 1/sqrt(p): the hardware estimate (about 23 bits) refined by one third-order
// step.  With e = 1 - p r^2, 1/sqrt(p) = r (1 - e)^(-1/2) = r (1 + e/2 + 3e^2/8
// + ...); the dropped terms are below 2^-66, so the result is within about
// one ulp.
__device__ __forceinline__ double rsq_refined(double p) {
    const double r = __builtin_amdgcn_rsq(p);
    const double e = fma(-p * r, r, 1.0);
    return fma(r * e, fma(e, 0.375, 0.5), r);
}

// Orders this lane's LDS writes before the other lanes' later reads within
// the wavefront (LDS operations of one wavefront complete in issue order).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

static constexpr int LTS = TB + 1;   // padded LDS row stride of the tile and the inverse
static constexpr int PB = 16;        // panel / block width inside the diagonal block
static constexpr int NPB = TB / PB;  // panels per diagonal block

// One 16 x 16 x 16 product on matrix cores for the calling wave:
// acc0 + acc1 += sgn * A B with A and B 16 x 16 blocks (row stride LTS) in
// LDS, the K steps alternating between the two accumulators so that two
// product chains are in flight; accumulator register r holds row lane/16 + 4r,
// column lane%16 (the v_mfma_f64_16x16x4f64 layout).
__device__ __forceinline__ void mma16(const double *__restrict__ Ab, const double *__restrict__ Bb, double sgn,
                                      d4 &acc0, d4 &acc1) {
    const int l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
#pragma unroll
    for (int kk = 0; kk < PB; kk += 8) {
        const double a0 = sgn * Ab[li * LTS + kk + lk], b0 = Bb[(kk + lk) * LTS + li];
        const double a1 = sgn * Ab[li * LTS + kk + 4 + lk], b1 = Bb[(kk + 4 + lk) * LTS + li];
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc1, 0, 0, 0);
    }
}

// The same with B given transposed: acc0 + acc1 += sgn * A C^T for 16 x 16
// blocks A and C (row stride LTS) in LDS.
__device__ __forceinline__ void mma16_nt(const double *__restrict__ Ab, const double *__restrict__ Cb, double sgn,
                                         d4 &acc0, d4 &acc1) {
    const int l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
#pragma unroll
    for (int kk = 0; kk < PB; kk += 8) {
        const double a0 = sgn * Ab[li * LTS + kk + lk], b0 = Cb[li * LTS + kk + lk];
        const double a1 = sgn * Ab[li * LTS + kk + 4 + lk], b1 = Cb[li * LTS + kk + 4 + lk];
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc1, 0, 0, 0);
    }
}

// X_qq = L_qq^-1 for the 16 x 16 diagonal block q of the factor in T, by one
// wave: lane c < 16 solves L_qq x = e_c by forward substitution, taking
// 1/L_rr from rd; the entries of column r + 1 are read from LDS while column
// r is applied.
__device__ __forceinline__ void inverse_diag_block(const double *__restrict__ T, double *__restrict__ X,
                                                   const double *__restrict__ rd, int q) {
    const int l = threadIdx.x & 63, c = l & 15;
    const int b0 = PB * q;
    double rdv[PB];
#pragma unroll
    for (int r = 0; r < PB; r++) rdv[r] = rd[b0 + r];
    double x[PB];
#pragma unroll
    for (int r = 0; r < PB; r++) x[r] = (r == c) ? 1.0 : 0.0;
    double lc[PB];
#pragma unroll
    for (int s = 1; s < PB; s++) lc[s] = T[(b0 + s) * LTS + b0];
#pragma unroll
    for (int r = 0; r < PB; r++) {
        double ln[PB];
        if (r + 1 < PB) {
#pragma unroll
            for (int s = r + 2; s < PB; s++) ln[s] = T[(b0 + s) * LTS + b0 + r + 1];
        }
        x[r] *= rdv[r];
#pragma unroll
        for (int s = r + 1; s < PB; s++) x[s] = fma(-lc[s], x[r], x[s]);
        if (r + 1 < PB) {
#pragma unroll
            for (int s = r + 2; s < PB; s++) lc[s] = ln[s];
        }
    }
    if (l < PB) {
#pragma unroll
        for (int r = 0; r < PB; r++) X[(b0 + r) * LTS + b0 + l] = x[r];
    }
}

// X_qj = -X_qq sum_{k=j}^{q-1} L_qk X_kj for the column blocks j in [jb, je)
// of row block q, by one wave on matrix cores (X_qq and the row blocks of X
// above q must be complete).
__device__ __forceinline__ void inverse_off_blocks(const double *__restrict__ T, double *__restrict__ X, int q,
                                                   int jb, int je) {
    const int l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
    const int b0 = PB * q;
    for (int j = jb; j < je; j++) {
        d4 s0 = {0.0, 0.0, 0.0, 0.0}, s1 = s0;
        for (int k = j; k < q; k++) mma16(T + b0 * LTS + PB * k, X + PB * k * LTS + PB * j, 1.0, s0, s1);
        // the accumulator of S is already in the B operand layout
        const d4 s = s0 + s1;
        d4 o0 = {0.0, 0.0, 0.0, 0.0}, o1 = o0;
#pragma unroll
        for (int r = 0; r < 4; r += 2) {
            const double a0 = -X[(b0 + li) * LTS + b0 + 4 * r + lk];
            const double a1 = -X[(b0 + li) * LTS + b0 + 4 * r + 4 + lk];
            o0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, s[r], o0, 0, 0, 0);
            o1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, s[r + 1], o1, 0, 0, 0);
        }
        const d4 o = o0 + o1;
#pragma unroll
        for (int r = 0; r < 4; r++) X[(b0 + lk + 4 * r) * LTS + PB * j + li] = o[r];
    }
}

// Store, by one wave, the panel's rows of the forward result and (store_L)
// the finished columns of panel pp (the lower triangle of the nb x nb block
// within them).
__device__ __forceinline__ void write_panel_L(const double *__restrict__ T, const double *__restrict__ yv,
                                              double *__restrict__ A, double *__restrict__ y, int64_t n, int64_t k0,
                                              int nb, int pp, int lane, bool store_L) {
    const int c = PB * pp + (lane & 15);
    if (store_L) {
#pragma unroll 4
        for (int r = PB * pp + (lane >> 4); r < nb; r += 4)
            if (c <= r) A[(k0 + r) * n + k0 + c] = T[r * LTS + c];
    }
    if (lane < PB && PB * pp + lane < nb) y[PB * pp + lane] = yv[PB * pp + lane];
}

// Store, by one wave, row block q of the inverse (64 columns, zero above the
// diagonal block).
__device__ __forceinline__ void write_inverse_rows(const double *__restrict__ X, double *__restrict__ linv, int q,
                                                   int lane) {
#pragma unroll
    for (int r = PB * q; r < PB * (q + 1); r++)
        linv[r * TB + lane] = (lane < PB * (q + 1)) ? X[r * LTS + lane] : 0.0;
}

// Element (r, c) of a diagonal tile into the LDS layout the factor expects:
// the lower triangle in place and, inside the 16 x 16 diagonal blocks, its
// mirror in the upper one (identity outside the nb x nb block).  Stores with
// nothing to write go to the unused padding column.
__device__ __forceinline__ void put_diag_elem(double *__restrict__ T, int r, int c, int nb, double v) {
    const double e = (r < nb && c < nb) ? v : (r == c ? 1.0 : 0.0);
    const bool same = (r / PB) == (c / PB);
    T[(c > r && same) ? r * LTS + TB : r * LTS + c] = e;
    T[(c < r && same) ? c * LTS + r : r * LTS + TB] = e;
}

// Factor one 64 x 64 diagonal block (A_kk = L L^T), forward-substitute its
// slice of the right-hand side (y = L^-1 b) and invert the factor
// (X = L^-1), with four wavefronts and the tile held in LDS, blocked by
// 16 x 16 blocks:
//  - factorization, right-looking by 16-column panels.  Wave 0 factors a
//    panel with lane r holding row r's 16 panel entries in registers.  The
//    pivot's column is taken from row pr of lane pr (the panel's diagonal
//    block is read symmetrically from the lower triangle), broadcast through
//    scalar registers in one batch per pivot, and the next pivot is formed
//    from broadcast values as soon as 1/sqrt of the current one is known.  The
//    update of a row uses w_r = L_r,pr / L_pr,pr against the unscaled pivot
//    row (one fma per entry); the right-hand side is carried the same way and
//    scaled once at the end of the panel.  Then the panel's rank-16 update of
//    the trailing blocks runs on matrix cores (one 16 x 16 block per wave at a
//    time);
//  - inverse, by 16 x 16 blocks, one and two panels behind the factorization:
//    while wave 0 factors panel p, wave 1 inverts diagonal block p - 1 and
//    wave 2 forms the off-diagonal blocks of row block p - 2 on matrix cores
//    (X_qj = -X_qq sum_k L_qk X_kj); what is left follows the last panel;
//  - finished panels, right-hand side rows and inverse row blocks are stored
//    by wave 3 while the factorization goes on.
// Only the lower triangle of the tile is read; the 16 x 16 diagonal blocks are
// mirrored in LDS and kept in both triangles by the trailing updates, so a
// panel reads its rows straight from the tile.
// The block is held in T (layout of put_diag_elem) with the right-hand side
// slice in yv; X, rdiag, pvs and sfail are LDS work space (sfail zero on
// entry).  The caller has synchronised after filling them.  Writes y to
// y[0..nb), L^-1 (64 x 64, zero above the diagonal) to linv and, with
// store_L, the lower triangle of L to the block at A[k0.., k0..] (row stride
// n; no later step reads it: the solves use L^-1).  Returns 0,
// or the 1-based row index of a pivot that is not a positive normal number:
// the factorization stops there (the caller records it as prm.info; the
// panels stored before it are left in the work buffer, which no later kernel
// reads once info is set).
__device__ __forceinline__ int factor_diag_tile(double *__restrict__ T, double *__restrict__ X,
                                                double *__restrict__ yv, double *__restrict__ rdiag,
                                                double *__restrict__ pvs, int &sfail, double *__restrict__ A,
                                                int64_t n, int64_t k0, int nb, double *__restrict__ y,
                                                double *__restrict__ linv, bool store_L) {
    const int t = threadIdx.x;
    const int w = t >> 6;
    const int i = t & 63;
#pragma unroll 1
    for (int p = 0; p < NPB; p++) {
        const int c0 = PB * p;
        if (w == 0) {
            // row i of the panel (the diagonal blocks are kept in both triangles)
            double a[PB];
#pragma unroll
            for (int k = 0; k < PB; k++) a[k] = T[i * LTS + c0 + k];
            double bi = yv[i];
            double pv = bcast(a[0], c0);
            double s[PB];
#pragma unroll
            for (int k = 1; k < PB; k++) s[k] = bcast(a[k], c0);
            double dn = bcast(a[1], c0 + 1);
            double bpr = bcast(bi, c0);
#pragma unroll
            for (int j = 0; j < PB; j++) {
                const int pr = c0 + j;
                const double rj = rsq_refined(pv);
                double pv_next = 0.0;
                if (j + 1 < PB) pv_next = fma(-(s[j + 1] * rj) * rj, s[j + 1], dn);
                const double lij = (i == pr) ? pv * rj : a[j] * rj;
                const double wv = (i > pr) ? lij * rj : 0.0;
                a[j] = lij;
#pragma unroll
                for (int k = j + 1; k < PB; k++) a[k] = fma(-wv, s[k], a[k]);
                bi = fma(-wv, bpr, bi);
                // rows above pr land in the unused upper triangle
                T[i * LTS + pr] = lij;
                rdiag[pr] = rj;
                pvs[pr] = pv;
                if (j + 1 < PB) {
#pragma unroll
                    for (int k = j + 2; k < PB; k++) s[k] = bcast(a[k], pr + 1);
                    if (j + 2 < PB) dn = bcast(a[j + 2], pr + 2);
                    bpr = bcast(bi, pr + 1);
                    pv = pv_next;
                }
            }
            wave_sync();
            // the panel's pivots checked at once; rows of the panel get
            // y = residual / L_ii, the rows below keep their residual
            const double pl = pvs[c0 + (i & 15)];
            const bool bad = (i < PB) && !(pl >= 2.2250738585072014e-308 && pl <= 1.7976931348623157e308);
            const unsigned long long bm = __ballot(bad);
            if (i == 0 && bm) sfail = (int)(k0 + c0 + __builtin_ctzll(bm) + 1);
            if (i >= c0) yv[i] = (i < c0 + PB) ? bi * rdiag[i] : bi;
        } else if (w == 1 && p >= 1) {
            inverse_diag_block(T, X, rdiag, p - 1);
        } else if (w == 2 && p >= 2) {
            inverse_off_blocks(T, X, p - 2, 0, p - 2);
        } else if (w == 3 && p >= 1) {
            // finished parts go out while the factorization continues: the
            // columns and right-hand side rows of the previous panel, and the
            // row block of the inverse completed two panels ago
            write_panel_L(T, yv, A, y, n, k0, nb, p - 1, i, store_L);
            if (p >= 3) write_inverse_rows(X, linv, p - 3, i);
        }
        __syncthreads();
        if (sfail) return sfail;
        // rank-16 update of the trailing blocks (I >= J > p) on matrix cores
        const int nt = NPB - 1 - p;
        const int nblk = nt * (nt + 1) / 2;
        for (int b = w; b < nblk; b += 4) {
            int bi_ = 0;
            while ((bi_ + 1) * (bi_ + 2) / 2 <= b) bi_++;
            const int bj = b - bi_ * (bi_ + 1) / 2;
            const int R = c0 + PB * (1 + bi_), Cc = c0 + PB * (1 + bj);
            const int li = i & 15, lk = i >> 4;
            d4 acc0, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int r = 0; r < 4; r++) acc0[r] = T[(R + lk + 4 * r) * LTS + Cc + li];
            mma16_nt(T + R * LTS + c0, T + Cc * LTS + c0, -1.0, acc0, acc1);
            const d4 acc = acc0 + acc1;
#pragma unroll
            for (int r = 0; r < 4; r++) T[(R + lk + 4 * r) * LTS + Cc + li] = acc[r];
        }
        if (nblk > 0) __syncthreads();
    }
    // the rest of the inverse: diagonal block 3 (wave 0) and the two
    // off-diagonal blocks of row block 2 (waves 1, 2), then those of row
    // block 3, one per wave; wave 3 writes the last panel meanwhile
    if (w == 0) inverse_diag_block(T, X, rdiag, NPB - 1);
    else if (w == 1) inverse_off_blocks(T, X, NPB - 2, 1, 2);
    else if (w == 2) inverse_off_blocks(T, X, NPB - 2, 0, 1);
    else write_panel_L(T, yv, A, y, n, k0, nb, NPB - 1, i, store_L);
    __syncthreads();
    if (w < NPB - 1) inverse_off_blocks(T, X, NPB - 1, w, w + 1);
    else write_inverse_rows(X, linv, 1, i);
    __syncthreads();
    // row blocks 2 and 3 of the inverse (zero above the diagonal blocks)
#pragma unroll
    for (int u = 0; u < 2 * PB * TB / 256; u++) {
        const int e = t + 256 * u;
        const int r = 2 * PB + (e >> 6), c = e & 63;
        linv[r * TB + c] = (r / PB >= c / PB) ? X[r * LTS + c] : 0.0;
    }
    return 0;
}

__global__ __launch_bounds__(256) void k_potf2(const DenseDesc *__restrict__ desc, DenseParam *__restrict__ prm,
                                               double *__restrict__ work, int step) {
    __shared__ __align__(16) double T[TB * LTS];
    __shared__ __align__(16) double X[TB * LTS];
    __shared__ double yv[TB];
    __shared__ double rdiag[TB];
    __shared__ double pvs[TB];
    __shared__ int sfail;
    const int m = blockIdx.y;
    const DenseParam pm = prm[m];
    const DenseDesc d = desc[m];
    if (!pm.active || pm.info) return;
    const int64_t k0 = (int64_t)TB * step;
    if (k0 >= d.n) return;
    const int nb = (int)std::min<int64_t>(TB, d.n - k0);
    double *A = work + d.a_off;
    const int t = threadIdx.x;
    const int w = t >> 6;
    const int i = t & 63;
    {   // the tile; only its lower triangle is read.  The loads are
        // unconditional from a clamped in-bounds address so that all of them
        // are in flight at once.
        double v[TB / 4];
        const int ci = std::min(i, nb - 1);
#pragma unroll
        for (int u = 0; u < TB / 4; u++) {
            const int r = std::min(w + 4 * u, nb - 1);
            v[u] = A[(k0 + r) * d.n + k0 + ci];
        }
#pragma unroll
        for (int u = 0; u < TB / 4; u++) put_diag_elem(T, w + 4 * u, i, nb, v[u]);
    }
    if (t < TB) yv[t] = work[d.v_off + k0 + std::min(t, nb - 1)] * (t < nb ? 1.0 : 0.0);
    if (t == 0) sfail = 0;
    __syncthreads();
    const int f = factor_diag_tile(T, X, yv, rdiag, pvs, sfail, A, d.n, k0, nb, work + d.v_off + k0,
                                   work + d.linv_off + (int64_t)step * TB * TB, true);
    if (f && t == 0 && f <= d.n) prm[m].info = f;
}

// Panel solve on matrix cores: rows below block `step`:  P <- P L_kk^-T,
// then b_rows -= P y_k (forward substitution).
__global__ __launch_bounds__(256) void k_trsm(const DenseDesc *__restrict__ desc, const DenseParam *__restrict__ prm,
                                              double *__restrict__ work, int step) {
    // one staging buffer: the two K chunks during the product, then the result tile
    __shared__ double sm[2 * TB * LDK];
    __shared__ double yk[TB];
    double *As = sm, *Bs = sm + TB * LDK;
    double(*Ts)[TB + 1] = (double(*)[TB + 1])sm;
    const int m = blockIdx.y;
    const DenseDesc d = desc[m];
    if (!prm[m].active || prm[m].info) return;
    const int64_t k0 = (int64_t)TB * step;
    const int64_t R0 = k0 + TB + (int64_t)TB * blockIdx.x;
    if (R0 >= d.n) return;
    double *A = work + d.a_off;
    const double *linv = work + d.linv_off + (int64_t)step * TB * TB;
    d4 acc[2][2];
    tile_gemm_nt(As, Bs, A, d.n, R0, k0, d.n, k0 + TB, linv, TB, 0, 0, TB, TB, acc);
    const int64_t nrow = std::min<int64_t>(TB, d.n - R0);
#pragma unroll
    for (int rb = 0; rb < 2; rb++)
#pragma unroll
        for (int cb = 0; cb < 2; cb++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int row = ACC_ROW(rb, r), col = ACC_COL(cb);
                Ts[row][col] = acc[rb][cb][r];
                if (row < nrow) A[(R0 + row) * d.n + k0 + col] = acc[rb][cb][r];
            }
    if (threadIdx.x < TB) yk[threadIdx.x] = work[d.v_off + k0 + threadIdx.x];
    __syncthreads();
    if (threadIdx.x < nrow) {
        double s = 0.0;
        for (int c = 0; c < TB; c++) s += Ts[threadIdx.x][c] * yk[c];
        work[d.v_off + R0 + threadIdx.x] -= s;
    }
}

// Trailing update on matrix cores: C_IJ -= P_I P_J^T for tiles I >= J.
// Symmetric update on matrix cores of the lower tiles of a region:
// A[r][c] -= sum_k L[r][k] L[c][k] over the K columns [k0, k0 + kw), for
// rows r >= T0 and columns T0 <= c < Cend (64x64 tiles, I >= J).  A panel
// step updates only the rest of its panel (narrow column range); the update
// after a panel covers the whole trailing matrix with the panel's width as K.
__global__ __launch_bounds__(256) void k_syrk(const DenseDesc *__restrict__ desc, const DenseParam *__restrict__ prm,
                                              double *__restrict__ work, int kstep, int kw, int tstep, int cend_step) {
    __shared__ double sm[2 * TB * LDK];
    double *As = sm, *Bs = sm + TB * LDK;
    const int m = blockIdx.y;
    const DenseDesc d = desc[m];
    if (!prm[m].active || prm[m].info) return;
    const int64_t k0 = (int64_t)TB * kstep;
    const int64_t T0 = (int64_t)TB * tstep;
    if (T0 >= d.n) return;
    const int64_t cend = std::min<int64_t>((int64_t)TB * cend_step, d.n);
    const int64_t ntr = (d.n - T0 + TB - 1) / TB;            // tile rows
    const int64_t ntc = (cend - T0 + TB - 1) / TB;           // tile columns
    if (ntc <= 0) return;
    const int64_t idx = blockIdx.x;
    int64_t I, J;
    if (ntc == ntr) {   // whole lower triangle: idx = I (I + 1) / 2 + J
        if (idx >= ntr * (ntr + 1) / 2) return;
        I = (int64_t)((sqrt(8.0 * (double)idx + 1.0) - 1.0) * 0.5);
        while (I * (I + 1) / 2 > idx) I--;
        while ((I + 1) * (I + 2) / 2 <= idx) I++;
        J = idx - I * (I + 1) / 2;
    } else {            // a few tile columns: column J holds tile rows J..ntr-1
        int64_t r = idx;
        J = 0;
        while (J < ntc && r >= ntr - J) {
            r -= ntr - J;
            J++;
        }
        if (J >= ntc) return;
        I = J + r;
    }
    const int64_t ri = T0 + TB * I, rj = T0 + TB * J;
    const int64_t kend = std::min<int64_t>(k0 + kw, d.n);
    double *A = work + d.a_off;
    d4 acc[2][2];
    tile_gemm_nt(As, Bs, A, d.n, ri, k0, d.n, kend, A, d.n, rj, k0, d.n, kend, acc, kw);
#pragma unroll
    for (int rb = 0; rb < 2; rb++)
#pragma unroll
        for (int cb = 0; cb < 2; cb++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int64_t row = ri + ACC_ROW(rb, r), col = rj + ACC_COL(cb);
                if (row < d.n && col < cend) A[row * d.n + col] -= acc[rb][cb][r];
            }
}

// Backward substitution, R block rows per launch: rows k, k-1, ..., k-R+1
// (those >= 0 that the matrix has; k = `step`).  Every workgroup forms the
// rows' solutions in order, x_r = L_rr^-T (y_r - sum of L_r'r^T x_r' over the
// rows r' above r in the group), and workgroup J below the group applies
// y_J <- y_J - sum_r L_rJ^T x_r (rows in order); workgroup 0 stores x.  All
// tiles are loaded before the first product.  Four threads share each
// 64-term dot product.
template <int R>
__global__ __launch_bounds__(256) void k_backsub_rows(const DenseDesc *__restrict__ desc,
                                                      const DenseParam *__restrict__ prm, double *__restrict__ work,
                                                      double *__restrict__ x, const int64_t *__restrict__ x_off,
                                                      int step) {
    __shared__ double xs[R][TB], ys[R][TB];
    const int m = blockIdx.y;
    const DenseDesc d = desc[m];
    if (!prm[m].active || prm[m].info) return;
    const int lo = step - R + 1;   // lowest row of the group (may be < 0)
    if ((int64_t)TB * std::max(lo, 0) >= d.n) return;   // the group lies beyond this (smaller) matrix
    const int64_t J = blockIdx.x;
    if (J > 0 && J >= lo) return;
    const bool upd = J < lo;
    const int t = threadIdx.x, o = t >> 2, part = t & 3;
    const double *A = work + d.a_off;
    int nb[R];
#pragma unroll
    for (int i = 0; i < R; i++) {
        const int64_t r0 = (int64_t)TB * (step - i);
        nb[i] = (step - i >= 0 && r0 < d.n) ? (int)std::min<int64_t>(TB, d.n - r0) : 0;
    }
    double li[R][16], lj[R][16], lc[R > 1 ? R * (R - 1) / 2 : 1][16];
#pragma unroll
    for (int i = 0; i < R; i++) {
        const int64_t r0 = (int64_t)TB * (step - i);
#pragma unroll
        for (int q = 0; q < 16; q++) {
            const int r = part + 4 * q;
            li[i][q] = nb[i] ? work[d.linv_off + (int64_t)(step - i) * TB * TB + r * TB + o] : 0.0;
            lj[i][q] = (upd && r < nb[i]) ? A[(r0 + r) * d.n + TB * J + o] : 0.0;
        }
    }
    // lc[p(i, i')]: the tile (row block step - i', column block step - i), i' < i
#pragma unroll
    for (int i = 1; i < R; i++)
#pragma unroll
        for (int ip = 0; ip < i; ip++) {
            const int p = i * (i - 1) / 2 + ip;
            const int64_t r0 = (int64_t)TB * (step - ip), c0 = (int64_t)TB * (step - i);
#pragma unroll
            for (int q = 0; q < 16; q++) {
                const int r = part + 4 * q;
                lc[p][q] = (nb[i] && r < nb[ip]) ? A[(r0 + r) * d.n + c0 + o] : 0.0;
            }
        }
    if (t < TB) {
#pragma unroll
        for (int i = 0; i < R; i++)
            ys[i][t] = t < nb[i] ? work[d.v_off + (int64_t)TB * (step - i) + t] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < R; i++) {
        if (i > 0) {   // y_i -= L_i'i^T x_i' for the rows above, in order
            double yi = ys[i][o];
#pragma unroll
            for (int ip = 0; ip < i; ip++) {
                const int p = i * (i - 1) / 2 + ip;
                double sum = 0.0;
#pragma unroll
                for (int q = 0; q < 16; q++) sum += lc[p][q] * xs[ip][part + 4 * q];
                sum += __shfl_xor(sum, 1, 64);
                sum += __shfl_xor(sum, 2, 64);
                yi -= sum;
            }
            __syncthreads();
            if (part == 0) ys[i][o] = yi;
            __syncthreads();
        }
        double sum = 0.0;   // x_i[o] = sum_c Linv_i[c][o] y_i[c]
#pragma unroll
        for (int q = 0; q < 16; q++) sum += li[i][q] * ys[i][part + 4 * q];
        sum += __shfl_xor(sum, 1, 64);
        sum += __shfl_xor(sum, 2, 64);
        if (part == 0) xs[i][o] = sum;
        __syncthreads();
        if (J == 0 && t < nb[i]) x[x_off[m] + (int64_t)TB * (step - i) + t] = xs[i][t];
    }
    if (!upd) return;
    double yJ = 0.0;   // y_J[o] <- ((y_J[o] - L_0J^T x_0) - L_1J^T x_1) - ...
#pragma unroll
    for (int i = 0; i < R; i++) {
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < 16; q++) sum += lj[i][q] * xs[i][part + 4 * q];
        sum += __shfl_xor(sum, 1, 64);
        sum += __shfl_xor(sum, 2, 64);
        if (i == 0) yJ = work[d.v_off + TB * J + o];
        yJ -= sum;
    }
    if (part == 0) work[d.v_off + TB * J + o] = yJ;
}

// ---------------------------------------------------------------- dataflow factorization
// One persistent launch factors a set of damped matrices and forward-
// substitutes their right-hand sides (A = L L^T, y = L^-1 b, and L_kk^-1 per
// diagonal block for the back substitution), with the same 64 x 64 tiles as
// the launch-per-step path.  Work is taken from one queue by running workgroups
// (an atomic ticket), in this order:
//  - one walker per matrix.  For j = 0, 1, ... it takes the diagonal tile's
//    partial sum P_jj = A_jj - sum_{k<j-1} L_jk L_jk^T, subtracts the last
//    term L_j,j-1 L_j,j-1^T (held in LDS from its previous step), factors and
//    inverts the block (factor_diag_tile), then solves the tile below,
//    L_j+1,j = P_j+1,j L_jj^-T, with the inverse still in LDS.  Only the
//    walker's work lies on the critical path, and it never waits for a
//    launch boundary;
//  - by column c = 0, 1, ...: tile tasks L_ic = (A_ic - sum_{k<c} L_ik L_ck^T)
//    L_cc^-T for i >= c + 3, then the two partial sums of row r = c + 2 that
//    the walker takes at its steps r - 1 and r, each left in place: P_rr with
//    the right-hand side rows b_r - sum_{k<=c} L_rk y_k, and P_r,r-1 =
//    A_r,r-1 - sum_{k<=c} L_rk L_r-1,k^T.  Both tasks form L_rc themselves
//    (the same arithmetic, so the same bits), beside their partial sums and
//    from the raw tile (r, c) they load first; the off-diagonal task stores
//    and publishes it once the diagonal task has read the raw tile.
// The raw tiles come straight from the undamped matrix H (damped on the
// diagonal as they are loaded, A = H + mu max(diag H, floor)) and the raw
// right-hand side from g (b = -g): each is read once, by the task that first
// uses it, and no damped copy is made.  Partial sums and L go to the work
// matrix.  A task accumulates its sums over k in order as the tiles L_.k
// become final, so each result is formed in a fixed order whatever the
// schedule.
// Completion is published with per-tile flags: every thread's stores, an
// agent-scope release fence (written back from the XCD's L2), then the flag;
// a consumer polls the flag and takes an agent-scope acquire fence before
// reading.  A task waits only for tasks earlier in the queue, and a task is
// taken only by a running workgroup, so the earliest unfinished task can
// always proceed.  Every wait is bounded: after `limit` polls the launch is
// aborted (all waits end, prm.info = -1 for the matrices not finished);
// a pivot failure abandons the matrix (prm.info as in k_potf2).
struct FlowTask {
    int32_t m, kind, i, c;
};
static constexpr int FLOW_WALK = 0, FLOW_TILE = 1, FLOW_PDIAG = 2, FLOW_POFF = 3;
static constexpr int FLOW_MAX_MATS = 128;     // walkers per launch
static constexpr int32_t FLOW_MAX_N = 6144;   // larger matrices take the launch-per-step path
static constexpr int FLOW_SPIN = 1 << 20;     // polls before a wait gives up (each about 1 us)

// Flags of one matrix with T tile rows: T*T tile flags (i, k), T diagonal
// flags, 3 T flags of the partial-sum tasks and one "abandoned" flag.
__host__ __device__ static inline int64_t flow_flag_ints(int64_t T) { return T * T + 4 * T + 1; }

// Pointers with their address space spelled out: the task bodies below are
// compiled out of line (each with its own register allocation), and their
// LDS and global accesses must still compile to ds_ and global_ instructions.
typedef __attribute__((address_space(3))) double lds_f64;
typedef __attribute__((address_space(3))) int lds_i32;
typedef __attribute__((address_space(1))) double glb_f64;
typedef __attribute__((address_space(1))) int glb_i32;

struct FlowMat {
    glb_i32 *fl;   // fl[i * T + k]: tile (i, k) of L final
    glb_i32 *dg;   // dg[k]: diagonal block k factored; its inverse and y rows final
    glb_i32 *po;   // po[r]: partial sum of tile (r, r - 1) in place
    glb_i32 *pd;   // pd[r]: partial sums of tile (r, r) and of rows r of b in place
    glb_i32 *ra;   // ra[r]: raw tile (r, r - 2) read by the diagonal task
    glb_i32 *ab;   // matrix abandoned
    int T;
};

__device__ __forceinline__ int flag_get(glb_i32 *f) {
    return __hip_atomic_load((int *)f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void flag_set(glb_i32 *f, int order) {
    if (order == __ATOMIC_RELEASE)
        __hip_atomic_store((int *)f, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    else
        __hip_atomic_store((int *)f, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0: polls *f until it is set.  False if the matrix was abandoned, the
// launch aborted, or `limit` polls went by (which aborts the launch); a
// negative limit gives up at once.
__device__ __forceinline__ bool flow_poll(glb_i32 *f, glb_i32 *ab, glb_i32 *gab, int limit) {
    if (limit < 0) {
        flag_set(gab, __ATOMIC_RELAXED);
        return false;
    }
    for (int it = 0;; it++) {
        if (flag_get(f)) return true;
        if (flag_get(ab) || flag_get(gab)) return false;
        if (it >= limit) {
            flag_set(gab, __ATOMIC_RELAXED);
            return false;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

// All threads: waits until *f is set; false on abandon or abort.
__device__ __forceinline__ bool flow_wait(glb_i32 *f, glb_i32 *ab, glb_i32 *gab, int limit, lds_i32 *s_val) {
    __syncthreads();
    if (threadIdx.x == 0) {
        *s_val = flow_poll(f, ab, gab, limit) ? 1 : 0;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    return *s_val != 0;
}

// All threads: waits until the tiles (rows[q], klo) of L are final and
// returns the end of the run of columns k in [klo, kend) whose tiles
// (rows[q], k) all are; -1 on abandon or abort.
template <int NR>
__device__ __forceinline__ int flow_wait_cols(const FlowMat &fm, const int (&rows)[NR], int klo, int kend,
                                              glb_i32 *gab, int limit, lds_i32 *s_val) {
    __syncthreads();
    if (threadIdx.x == 0) {
        bool ok = true;
        for (int q = 0; q < NR && ok; q++) ok = flow_poll(fm.fl + rows[q] * fm.T + klo, fm.ab, gab, limit);
        int khi = -1;
        if (ok) {
            khi = klo + 1;
            for (; khi < kend; khi++) {
                bool all = true;
                for (int q = 0; q < NR; q++) all = all && flag_get(fm.fl + rows[q] * fm.T + khi) != 0;
                if (!all) break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *s_val = khi;
    }
    __syncthreads();
    return *s_val;
}

// All threads: makes this workgroup's stores visible at agent scope, then
// sets *f.
__device__ __forceinline__ void flow_publish(glb_i32 *f) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) flag_set(f, __ATOMIC_RELEASE);
}

// All threads: waits until *f1 and *f2 are set; false on abandon or abort.
__device__ __forceinline__ bool flow_wait2(glb_i32 *f1, glb_i32 *f2, glb_i32 *ab, glb_i32 *gab, int limit,
                                           lds_i32 *s_val) {
    __syncthreads();
    if (threadIdx.x == 0) {
        *s_val = (flow_poll(f1, ab, gab, limit) && flow_poll(f2, ab, gab, limit)) ? 1 : 0;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    return *s_val != 0;
}

// flow_publish of two flags behind one fence.
__device__ __forceinline__ void flow_publish2(glb_i32 *f1, glb_i32 *f2) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
        flag_set(f1, __ATOMIC_RELEASE);
        flag_set(f2, __ATOMIC_RELAXED);
    }
}

// Tile M[r0.., c0..] (row stride ld) into LDS S (row stride LTS), zero
// outside nr x nc; the loads are unconditional from clamped addresses.
__device__ __forceinline__ void tile_to_lds(double *__restrict__ S, const double *__restrict__ M, int64_t ld,
                                            int64_t r0, int64_t c0, int nr, int nc) {
    const int c = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int cc = min(c, nc - 1);
    double v[TB / 4];
#pragma unroll
    for (int u = 0; u < TB / 4; u++) v[u] = M[(r0 + min(w + 4 * u, nr - 1)) * ld + c0 + cc];
#pragma unroll
    for (int u = 0; u < TB / 4; u++) {
        const int r = w + 4 * u;
        S[r * LTS + c] = (r < nr && c < nc) ? v[u] : 0.0;
    }
}

// This thread's elements of tile M[r0.., c0..] in the accumulator layout,
// zero outside nr x nc.
__device__ __forceinline__ void tile_to_acc(d4 acc[2][2], const double *__restrict__ M, int64_t ld, int64_t r0,
                                            int64_t c0, int nr, int nc) {
    double v[16];
#pragma unroll
    for (int rb = 0; rb < 2; rb++)
#pragma unroll
        for (int cb = 0; cb < 2; cb++)
#pragma unroll
            for (int r = 0; r < 4; r++)
                v[8 * rb + 4 * cb + r] =
                    M[(r0 + min((int)ACC_ROW(rb, r), nr - 1)) * ld + c0 + min((int)ACC_COL(cb), nc - 1)];
#pragma unroll
    for (int rb = 0; rb < 2; rb++)
#pragma unroll
        for (int cb = 0; cb < 2; cb++)
#pragma unroll
            for (int r = 0; r < 4; r++)
                acc[rb][cb][r] = ((int)ACC_ROW(rb, r) < nr && (int)ACC_COL(cb) < nc) ? v[8 * rb + 4 * cb + r] : 0.0;
}

__device__ __forceinline__ void acc_to_global(const d4 acc[2][2], double *__restrict__ M, int64_t ld, int64_t r0,
                                              int64_t c0, int nr, int nc) {
#pragma unroll
    for (int rb = 0; rb < 2; rb++)
#pragma unroll
        for (int cb = 0; cb < 2; cb++)
#pragma unroll
            for (int r = 0; r < 4; r++)
                if ((int)ACC_ROW(rb, r) < nr && (int)ACC_COL(cb) < nc)
                    M[(r0 + ACC_ROW(rb, r)) * ld + c0 + ACC_COL(cb)] = acc[rb][cb][r];
}

// Into LDS (row stride LTS), rows >= nr cleared.
__device__ __forceinline__ void acc_to_lds(const d4 acc[2][2], double *__restrict__ S, int nr) {
#pragma unroll
    for (int rb = 0; rb < 2; rb++)
#pragma unroll
        for (int cb = 0; cb < 2; cb++)
#pragma unroll
            for (int r = 0; r < 4; r++)
                S[ACC_ROW(rb, r) * LTS + ACC_COL(cb)] = ((int)ACC_ROW(rb, r) < nr) ? acc[rb][cb][r] : 0.0;
}

__device__ __forceinline__ void acc_sub(d4 a[2][2], const d4 b[2][2]) {
#pragma unroll
    for (int rb = 0; rb < 2; rb++)
#pragma unroll
        for (int cb = 0; cb < 2; cb++) a[rb][cb] -= b[rb][cb];
}

__device__ __forceinline__ void acc_zero(d4 a[2][2]) {
#pragma unroll
    for (int rb = 0; rb < 2; rb++)
#pragma unroll
        for (int cb = 0; cb < 2; cb++) a[rb][cb] = d4{0.0, 0.0, 0.0, 0.0};
}

// acc += sgn P Q^T for 64 x 64 P and Q in LDS (row stride LTS), this wave's
// 32 x 32 quadrant.  LOWER: Q is block lower triangular by 16 x 16 blocks and
// its blocks above the diagonal hold stale data (read as zero).
template <bool LOWER>
__device__ __forceinline__ void mma64_nt(const double *__restrict__ P, const double *__restrict__ Q, double sgn,
                                         d4 acc[2][2]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r0 = 32 * (w >> 1), c0 = 32 * (w & 1);
    const int li = lane & 15, lk = lane >> 4;
#pragma unroll 4
    for (int kk = 0; kk < TB; kk += 4) {
        const int k = kk + lk;
        const double a0 = sgn * P[(r0 + li) * LTS + k], a1 = sgn * P[(r0 + 16 + li) * LTS + k];
        double b0 = Q[(c0 + li) * LTS + k], b1 = Q[(c0 + 16 + li) * LTS + k];
        if (LOWER) {
            b0 = (k / PB <= (c0 + li) / PB) ? b0 : 0.0;
            b1 = (k / PB <= (c0 + 16 + li) / PB) ? b1 : 0.0;
        }
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
}

// This thread's share of row t/4 of S y (64 x 64 S in LDS, row stride LTS;
// the four threads of a row take every fourth column).
__device__ __forceinline__ double lds_gemv_part(const double *__restrict__ S, const double *__restrict__ y) {
    const int row = threadIdx.x >> 2, part = threadIdx.x & 3;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < TB / 4; q++) s = fma(S[row * LTS + part + 4 * q], y[part + 4 * q], s);
    return s;
}

__device__ __forceinline__ double row_sum4(double s) {
    s += __shfl_xor(s, 1, 64);
    s += __shfl_xor(s, 2, 64);
    return s;
}

// acc += L_i. L_i.^T over the columns [ka, ka + kw) (kw a multiple of 32) of
// the tile row at ra, and this thread's share of L_i. y over the same columns
// (q, as in lds_gemv_part).  The next K chunk is loaded while the current one
// is used.
__device__ __forceinline__ void tile_syrk_y(double *__restrict__ lds, const double *__restrict__ A, int64_t n,
                                            int64_t ra, int64_t ka, int kw, const double *__restrict__ y,
                                            d4 acc[2][2], double &q) {
    double *As = lds, *ys = lds + TB * LDK;
    const int t = threadIdx.x, row = t >> 2, part = t & 3;
    double va[8], vy = 0.0;
    load_chunk(va, A, n, ra, ka, n, n);
    if (t < 32) vy = y[ka + t];
    for (int kc = 0; kc < kw; kc += 32) {
        store_chunk(As, va);
        if (t < 32) ys[t] = vy;
        __syncthreads();
        if (kc + 32 < kw) {
            load_chunk(va, A, n, ra, ka + kc + 32, n, n);
            if (t < 32) vy = y[ka + kc + 32 + t];
        }
        mma_chunk(As, As, acc);
#pragma unroll
        for (int e = 0; e < 8; e++) q = fma(As[row * LDK + part + 4 * e], ys[part + 4 * e], q);
        __syncthreads();
    }
}

// ---- the walker's tile products, shaped by their triangular operands
// A 64 x 64 diagonal tile by its ten lower 16 x 16 blocks (rb >= cb, taken
// in the order (0,0), (1,0), (1,1), (2,0), ..., (3,3)): wave w holds blocks
// w, w + 4 and (waves 0, 1) w + 8, each in the v_mfma_f64_16x16x4f64
// accumulator layout.
struct LowTile {
    d4 b[3];
};

__device__ __forceinline__ void low_block(int q, int &rb, int &cb) {
    rb = q >= 6 ? 3 : (q >= 3 ? 2 : (q >= 1 ? 1 : 0));
    cb = q - rb * (rb + 1) / 2;
}

// Loads the lower blocks of tile M[r0.., r0..] (row stride ld), zero outside
// nb x nb (loads from clamped addresses).
__device__ __forceinline__ void low_load(LowTile &D, const double *__restrict__ M, int64_t ld, int64_t r0, int nb) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
    double v[12];
#pragma unroll
    for (int s = 0; s < 3; s++) {
        int rb, cb;
        low_block(w + 4 * s, rb, cb);
        if (s == 2 && w >= 2) rb = cb = 0;
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int row = 16 * rb + lk + 4 * r, col = 16 * cb + li;
            v[4 * s + r] = M[(r0 + min(row, nb - 1)) * ld + r0 + min(col, nb - 1)];
        }
    }
#pragma unroll
    for (int s = 0; s < 3; s++) {
        int rb, cb;
        low_block(w + 4 * s, rb, cb);
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int row = 16 * rb + lk + 4 * r, col = 16 * cb + li;
            D.b[s][r] = (row < nb && col < nb) ? v[4 * s + r] : 0.0;
        }
    }
}

// The damped diagonal of a tile of H (as in damp_diag_tile).
__device__ __forceinline__ void low_damp(LowTile &D, double mu, double floor_) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int s = 0; s < 3; s++) {
        int rb, cb;
        low_block(w + 4 * s, rb, cb);
        if (rb != cb || (s == 2 && w >= 2)) continue;
#pragma unroll
        for (int r = 0; r < 4; r++)
            if (lk + 4 * r == li) {
                const double x = D.b[s][r];
                D.b[s][r] = x + mu * (x > floor_ ? x : floor_);
            }
    }
}

// D -= L L^T on the lower blocks, L (64 x 64) in LDS with row stride LTS.
__device__ __forceinline__ void low_syrk_sub(LowTile &D, const double *__restrict__ L) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int s = 0; s < 3; s++) {
        if (s == 2 && w >= 2) break;
        int rb, cb;
        low_block(w + 4 * s, rb, cb);
        d4 a0 = D.b[s], a1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < TB; kk += 8) {
            const double x0 = -L[(16 * rb + li) * LTS + kk + lk], y0 = L[(16 * cb + li) * LTS + kk + lk];
            const double x1 = -L[(16 * rb + li) * LTS + kk + 4 + lk], y1 = L[(16 * cb + li) * LTS + kk + 4 + lk];
            a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, y0, a0, 0, 0, 0);
            a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, y1, a1, 0, 0, 0);
        }
        D.b[s] = a0 + a1;
    }
}

// The lower blocks into the factor's LDS layout (put_diag_elem); the blocks
// above the diagonal are never read.
__device__ __forceinline__ void low_put(const LowTile &D, double *__restrict__ T, int nb) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int s = 0; s < 3; s++) {
        if (s == 2 && w >= 2) break;
        int rb, cb;
        low_block(w + 4 * s, rb, cb);
#pragma unroll
        for (int r = 0; r < 4; r++) put_diag_elem(T, 16 * rb + lk + 4 * r, 16 * cb + li, nb, D.b[s][r]);
    }
}

// L = P X^T for P (64 x 64) and X lower triangular (64 x 64, blocks above its
// diagonal blocks stale), both in LDS with row stride LTS: wave w forms row
// block w, each column block cb over k < 16 (cb + 1) only.  Element (cb, r)
// of this lane is row 16 w + lane/16 + 4 r, column 16 cb + lane%16.
struct RowTile {
    d4 c[4];
};

__device__ __forceinline__ void rows_trsm(const double *__restrict__ P, const double *__restrict__ X, RowTile &L) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int cb = 0; cb < 4; cb++) L.c[cb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < TB; kk += 4) {
        const double a = P[(16 * w + li) * LTS + kk + lk];
#pragma unroll
        for (int cb = kk / 16; cb < 4; cb++)
            L.c[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, X[(16 * cb + li) * LTS + kk + lk], L.c[cb], 0, 0, 0);
    }
}

__device__ __forceinline__ void rows_to_global(const RowTile &L, double *__restrict__ M, int64_t ld, int64_t r0,
                                               int64_t c0, int nr) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int cb = 0; cb < 4; cb++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int row = 16 * w + lk + 4 * r;
            if (row < nr) M[(r0 + row) * ld + c0 + 16 * cb + li] = L.c[cb][r];
        }
}

// Into LDS (row stride LTS), rows >= nr cleared.
__device__ __forceinline__ void rows_to_lds(const RowTile &L, double *__restrict__ S, int nr) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int cb = 0; cb < 4; cb++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int row = 16 * w + lk + 4 * r;
            S[row * LTS + 16 * cb + li] = row < nr ? L.c[cb][r] : 0.0;
        }
}

// Raw operands of one matrix: H (its row-major undamped block), g (its slice
// of the gradient) and the damping.
struct FlowRaw {
    glb_f64 *H;
    glb_f64 *g;
    double mu, floor_;
};

// A diagonal tile of H in the accumulator layout, damped on the diagonal
// as the damped system has it.
__device__ __forceinline__ void damp_diag_tile(d4 a[2][2], const FlowRaw &rw) {
#pragma unroll
    for (int rb = 0; rb < 2; rb++)
#pragma unroll
        for (int cb = 0; cb < 2; cb++)
#pragma unroll
            for (int r = 0; r < 4; r++)
                if (ACC_ROW(rb, r) == ACC_COL(cb)) {
                    const double v = a[rb][cb][r];
                    a[rb][cb][r] = v + rw.mu * (v > rw.floor_ ? v : rw.floor_);
                }
}

// L_ic = P L_cc^-T with P = raw - acc (raw: the tile A_ic as loaded): P
// and the inverse (from global) in LDS, the result in l (rows_trsm layout);
// the caller stores it.
__device__ __forceinline__ void flow_solve_tile(const d4 raw[2][2], int nr, const double *__restrict__ linv_c,
                                                const d4 acc[2][2], double *__restrict__ Pl, double *__restrict__ Xl,
                                                RowTile &l) {
    d4 p[2][2];
#pragma unroll
    for (int rb = 0; rb < 2; rb++)
#pragma unroll
        for (int cb = 0; cb < 2; cb++) p[rb][cb] = raw[rb][cb] - acc[rb][cb];
    acc_to_lds(p, Pl, nr);
    tile_to_lds(Xl, linv_c, TB, 0, 0, TB, TB);
    __syncthreads();
    rows_trsm(Pl, Xl, l);
}

// Diagonal partial task of row r = c + 2: P_rr = A_rr - sum_{k<=c} L_rk L_rk^T
// and b_r - sum_{k<=c} L_rk y_k, with L_rc formed here from the raw tile; the
// results go to the work matrix and right-hand side.
__device__ __noinline__ void flow_pdiag(const DenseDesc d, glb_f64 *gwork, const FlowRaw rw, const FlowMat fm, int r,
                                       int c, glb_i32 *gab, int limit, lds_f64 *glds, lds_i32 *s_val) {
    double *work = (double *)gwork, *lds = (double *)glds;
    const double *H = (const double *)rw.H, *g = (const double *)rw.g;
    const int64_t n = d.n;
    double *A = work + d.a_off, *v = work + d.v_off;
    const int64_t R0 = (int64_t)TB * r, C0 = (int64_t)TB * c;
    const int nr = (int)std::min<int64_t>(TB, n - R0);
    d4 raw[2][2], rrr[2][2];
    tile_to_acc(raw, H, n, R0, C0, nr, TB);
    tile_to_acc(rrr, H, n, R0, R0, nr, nr);
    damp_diag_tile(rrr, rw);
    const int row = threadIdx.x >> 2;
    const double graw = g[R0 + std::min(row, nr - 1)];
    flow_publish(fm.ra + r);   // the raw tile (r, c) is read
    d4 aa[2][2], ac[2][2];
    acc_zero(aa);
    acc_zero(ac);
    double q = 0.0;
    const int rows[2] = {r, c};
    for (int klo = 0; klo < c;) {
        const int khi = flow_wait_cols<2>(fm, rows, klo, c, gab, limit, s_val);
        if (khi < 0) return;
        const int64_t ka = (int64_t)TB * klo;
        tile_gemm_nt_acc(lds, lds + TB * LDK, A, n, R0, ka, n, n, A, n, C0, ka, n, n, aa, TB * (khi - klo));
        tile_syrk_y(lds, A, n, R0, ka, TB * (khi - klo), v, ac, q);
        klo = khi;
    }
    if (!flow_wait(fm.dg + c, fm.ab, gab, limit, s_val)) return;
    double *Pl = lds, *Xl = lds + TB * LTS, *ys = lds + 2 * TB * LTS;
    RowTile l;
    flow_solve_tile(raw, nr, work + d.linv_off + (int64_t)c * TB * TB, aa, Pl, Xl, l);
    __syncthreads();
    rows_to_lds(l, Pl, nr);
    if (threadIdx.x < TB) ys[threadIdx.x] = v[C0 + threadIdx.x];
    __syncthreads();
    mma64_nt<false>(Pl, Pl, 1.0, ac);
    q += lds_gemv_part(Pl, ys);
    acc_sub(rrr, ac);
    acc_to_global(rrr, A, n, R0, R0, nr, nr);
    q = row_sum4(q);
    if ((threadIdx.x & 3) == 0 && row < nr) v[R0 + row] = -graw - q;
    flow_publish(fm.pd + r);
}

// Off-diagonal partial task of row r = c + 2: L_rc (its sums formed beside
// those of the partial) and P_r,r-1 with the last term L_rc L_c+1,c^T (the
// walker's tile of step c), published behind one fence.
__device__ __noinline__ void flow_poff(const DenseDesc d, glb_f64 *gwork, const FlowRaw rw, const FlowMat fm, int r,
                                      int c, glb_i32 *gab, int limit, lds_f64 *glds, lds_i32 *s_val) {
    double *work = (double *)gwork, *lds = (double *)glds;
    const double *H = (const double *)rw.H;
    const int64_t n = d.n;
    double *A = work + d.a_off;
    const int64_t R0 = (int64_t)TB * r, C0 = (int64_t)TB * c, C1 = C0 + TB;
    const int nr = (int)std::min<int64_t>(TB, n - R0);
    d4 raw[2][2], rrp[2][2];
    tile_to_acc(raw, H, n, R0, C0, nr, TB);
    tile_to_acc(rrp, H, n, R0, C1, nr, TB);
    // L_rc goes to the tile (r, c) in place: first the diagonal task (earlier
    // in the queue) must have read the raw tile
    if (!flow_wait(fm.ra + r, fm.ab, gab, limit, s_val)) return;
    d4 aa[2][2], ab[2][2];
    acc_zero(aa);
    acc_zero(ab);
    const int rows[3] = {r, c, c + 1};
    for (int klo = 0; klo < c;) {
        const int khi = flow_wait_cols<3>(fm, rows, klo, c, gab, limit, s_val);
        if (khi < 0) return;
        const int64_t ka = (int64_t)TB * klo;
        tile_gemm_nt_acc(lds, lds + TB * LDK, A, n, R0, ka, n, n, A, n, C0, ka, n, n, aa, TB * (khi - klo));
        tile_gemm_nt_acc(lds, lds + TB * LDK, A, n, R0, ka, n, n, A, n, C1, ka, n, n, ab, TB * (khi - klo));
        klo = khi;
    }
    if (!flow_wait2(fm.dg + c, fm.fl + (c + 1) * fm.T + c, fm.ab, gab, limit, s_val)) return;
    double *Pl = lds, *Xl = lds + TB * LTS, *Ll = lds + 2 * TB * LTS;
    tile_to_lds(Ll, A, n, C1, C0, TB, TB);   // L_c+1,c, loaded beside the inverse
    RowTile l;
    flow_solve_tile(raw, nr, work + d.linv_off + (int64_t)c * TB * TB, aa, Pl, Xl, l);
    rows_to_global(l, A, n, R0, C0, nr);    // stored while the last term is formed
    __syncthreads();
    rows_to_lds(l, Pl, nr);
    __syncthreads();
    mma64_nt<false>(Pl, Ll, 1.0, ab);
    acc_sub(rrp, ab);
    acc_to_global(rrp, A, n, R0, C1, nr, TB);
    flow_publish2(fm.po + r, fm.fl + r * fm.T + c);
}

// Tile task: L_ic = (A_ic - sum_{k<c} L_ik L_ck^T) L_cc^-T for i >= c + 3.
__device__ __noinline__ void flow_tile(const DenseDesc d, glb_f64 *gwork, const FlowRaw rw, const FlowMat fm, int i,
                                      int c, glb_i32 *gab, int limit, lds_f64 *glds, lds_i32 *s_val) {
    double *work = (double *)gwork, *lds = (double *)glds;
    const double *H = (const double *)rw.H;
    const int64_t n = d.n;
    double *A = work + d.a_off;
    const int64_t R0 = (int64_t)TB * i, C0 = (int64_t)TB * c;
    const int nr = (int)std::min<int64_t>(TB, n - R0);
    d4 acc[2][2];
    acc_zero(acc);
    const int rows[2] = {i, c};
    for (int klo = 0; klo < c;) {
        const int khi = flow_wait_cols<2>(fm, rows, klo, c, gab, limit, s_val);
        if (khi < 0) return;
        const int64_t ka = (int64_t)TB * klo;
        tile_gemm_nt_acc(lds, lds + TB * LDK, A, n, R0, ka, n, n, A, n, C0, ka, n, n, acc, TB * (khi - klo));
        klo = khi;
    }
    d4 raw[2][2];
    tile_to_acc(raw, H, n, R0, C0, nr, TB);
    if (!flow_wait(fm.dg + c, fm.ab, gab, limit, s_val)) return;
    RowTile l;
    flow_solve_tile(raw, nr, work + d.linv_off + (int64_t)c * TB * TB, acc, lds, lds + TB * LTS, l);
    rows_to_global(l, A, n, R0, C0, nr);
    flow_publish(fm.fl + i * fm.T + c);
}

// Marks the matrix abandoned: a pivot failure (f > 0) or an aborted wait.
__device__ __forceinline__ void flow_abandon(glb_i32 *info, const FlowMat &fm, int f) {
    if (threadIdx.x == 0) {
        *info = f;
        flag_set(fm.ab, __ATOMIC_RELEASE);
    }
}

// Walker of one matrix (see above).  LDS: the factor's tile and inverse
// (lds, lds + TB * LTS), its vectors, and ybuf (y of the previous block).
// Step j factors D_j (held in dacc, b_j in bq), then waits once for both
// partial sums of block row j + 1, solves L_j+1,j while D_j+1 and b_j+1 load,
// forms their last terms, and publishes block j and that tile behind one
// fence.  L_jj itself is not stored.
__device__ __noinline__ void flow_walk(const DenseDesc d, glb_i32 *info, glb_f64 *gwork, const FlowRaw rw,
                                      const FlowMat fm, glb_i32 *gab, int limit, lds_f64 *glds, lds_f64 *gyv,
                                      lds_f64 *grdiag, lds_f64 *gpvs, lds_f64 *gybuf, lds_i32 *gsfail,
                                      lds_i32 *s_val) {
    double *work = (double *)gwork, *lds = (double *)glds, *yv = (double *)gyv, *rdiag = (double *)grdiag;
    const double *H = (const double *)rw.H, *g = (const double *)rw.g;
    double *pvs = (double *)gpvs, *ybuf = (double *)gybuf;
    int &sfail = *(int *)gsfail;
    const int64_t n = d.n;
    double *A = work + d.a_off, *v = work + d.v_off;
    double *Tl = lds, *Xl = lds + TB * LTS;
    const int t = threadIdx.x, row = t >> 2;
    // blocks 0 and 1 have no partial sums: raw tiles
    int nb = (int)std::min<int64_t>(TB, n);
    LowTile dt;
    low_load(dt, H, n, 0, nb);
    low_damp(dt, rw.mu, rw.floor_);
    double bq = (row < nb) ? -g[std::min(row, nb - 1)] : 0.0;
    for (int j = 0; j < fm.T; j++) {
        const int64_t k0 = (int64_t)TB * j;
        low_put(dt, Tl, nb);
        if ((t & 3) == 0) yv[row] = bq;
        if (t == 0) sfail = 0;
        __syncthreads();
        const int f = factor_diag_tile(Tl, Xl, yv, rdiag, pvs, sfail, A, n, k0, nb, v + k0,
                                       work + d.linv_off + (int64_t)j * TB * TB, false);
        if (f) {
            flow_abandon(info, fm, f);
            return;
        }
        __syncthreads();
        if (t < TB) ybuf[t] = yv[t];
        if (j + 1 >= fm.T) {
            flow_publish(fm.dg + j);
            break;
        }
        // partial sums of block row j + 1 (raw for j = 0)
        if (j >= 1 && !flow_wait2(fm.po + j + 1, fm.pd + j + 1, fm.ab, gab, limit, s_val)) {
            flow_abandon(info, fm, -1);
            return;
        }
        const int64_t r0 = k0 + TB;
        const int nr = (int)std::min<int64_t>(TB, n - r0);
        const double *Pj = j == 0 ? H : A;
        tile_to_lds(Tl, Pj, n, r0, k0, nr, TB);
        __syncthreads();
        // D_j+1 and b_j+1 are loaded while L_j+1,j = P_j+1,j L_jj^-T is formed
        // with the inverse in LDS
        low_load(dt, Pj, n, r0, nr);
        bq = (row < nr) ? (j == 0 ? -g[r0 + std::min(row, nr - 1)] : v[r0 + std::min(row, nr - 1)]) : 0.0;
        RowTile l;
        rows_trsm(Tl, Xl, l);
        rows_to_global(l, A, n, r0, k0, nr);
        __syncthreads();
        rows_to_lds(l, Xl, nr);
        __syncthreads();
        // the last terms of D_j+1 and b_j+1 (the stores of L_j+1,j complete
        // meanwhile), then block j and that tile are published
        if (j == 0) low_damp(dt, rw.mu, rw.floor_);
        low_syrk_sub(dt, Xl);
        bq -= row_sum4(lds_gemv_part(Xl, ybuf));
        flow_publish2(fm.dg + j, fm.fl + (j + 1) * fm.T + j);
        nb = nr;
    }
}

__global__ __launch_bounds__(256) void k_chol_flow(const DenseDesc *__restrict__ desc, DenseParam *__restrict__ prm,
                                                   const double *__restrict__ H, const int64_t *__restrict__ h_off,
                                                   const double *__restrict__ g, double *__restrict__ work,
                                                   const FlowTask *__restrict__ tasks,
                                                   int32_t n_tasks, int *__restrict__ flags,
                                                   const int64_t *__restrict__ fo, int *__restrict__ queue,
                                                   int *__restrict__ gab, int limit) {
    __shared__ __align__(16) double lds[3 * TB * LTS];
    __shared__ double yv[TB], rdiag[TB], pvs[TB], ybuf[TB];
    __shared__ int s_task, s_val, sfail;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_task = atomicAdd(queue, 1);
        __syncthreads();
        const int ti = s_task;
        if (ti >= n_tasks) return;
        const FlowTask tk = tasks[ti];
        const DenseParam pm = prm[tk.m];
        if (!pm.active || pm.info) continue;
        const DenseDesc d = desc[tk.m];
        const int T = (d.n + TB - 1) / TB;
        glb_i32 *fb = (glb_i32 *)(flags + fo[tk.m]);
        glb_i32 *fs = fb + T * T;
        const FlowMat fm{fb, fs, fs + T, fs + 2 * T, fs + 3 * T, fs + 4 * T, T};
        glb_f64 *gw = (glb_f64 *)work;
        const FlowRaw rw{(glb_f64 *)(H + h_off[tk.m]), (glb_f64 *)(g + 6LL * d.pose0), pm.mu, pm.floor_};
        glb_i32 *ga = (glb_i32 *)gab;
        lds_i32 *sv = (lds_i32 *)&s_val;
        if (tk.kind == FLOW_WALK)
            flow_walk(d, (glb_i32 *)&prm[tk.m].info, gw, rw, fm, ga, limit, (lds_f64 *)lds, (lds_f64 *)yv,
                      (lds_f64 *)rdiag, (lds_f64 *)pvs, (lds_f64 *)ybuf, (lds_i32 *)&sfail, sv);
        else if (tk.kind == FLOW_TILE)
            flow_tile(d, gw, rw, fm, tk.i, tk.c, ga, limit, (lds_f64 *)lds, sv);
        else if (tk.kind == FLOW_PDIAG)
            flow_pdiag(d, gw, rw, fm, tk.i, tk.c, ga, limit, (lds_f64 *)lds, sv);
        else
            flow_poff(d, gw, rw, fm, tk.i, tk.c, ga, limit, (lds_f64 *)lds, sv);
    }
}

// Task list of one matrix with T tile rows (the standalone solve): thread c
// writes the tasks of column c after the walker.
__global__ void k_flow_tasks_one(int32_t T, FlowTask *__restrict__ tasks) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c == 0) tasks[0] = FlowTask{0, FLOW_WALK, 0, 0};
    if (c >= T) return;
    int64_t o = 1;
    for (int cc = 0; cc < c; cc++) o += std::max(0, T - cc - 3) + (cc + 2 <= T - 1 ? 2 : 0);
    for (int i = c + 3; i < T; i++) tasks[o++] = FlowTask{0, FLOW_TILE, i, c};
    if (c + 2 <= T - 1) {
        tasks[o] = FlowTask{0, FLOW_PDIAG, c + 2, c};
        tasks[o + 1] = FlowTask{0, FLOW_POFF, c + 2, c};
    }
}

// ---------------------------------------------------------------- dataflow back substitution
// One launch solves L^T x = y for every matrix of a set, after the dataflow
// factorization (y = L^-1 b and the inverse diagonal blocks are in place).
// Task (m, p) owns block rows hi = T - 1 - 2p and lo = hi - 1 of matrix m (no
// lo at the top of an odd T).  Tasks are taken from a queue ticket in chain
// order (p-major), and task (m, p) waits for the flags of tasks (m, 0), ...,
// (m, p - 1) in turn, which hold earlier tickets: their workgroups are running
// or done, so the chain cannot deadlock.  Before each wait the task loads the
// four tiles of L that couple that pair of rows to its own, so the loads
// overlap the wait; it then subtracts L_kr^T x_k from y_r for k descending,
// as the two-row launches do.  With every update in, x_hi = L_hi^-T y_hi,
// y_lo -= L_(hi,lo)^T x_hi and x_lo = L_lo^-T y_lo, and one flag publishes
// both rows.  Each wait is bounded; a give-up marks the matrix failed
// (info = -1) and abandons its other tasks.
struct BsTask {
    int32_t m, p;
};

// (sum_q l[q] v[part + 4 q]) summed over the four parts of a column
__device__ __forceinline__ double bs_dot16(const double (&l)[16], const double *v, int part) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 16; q++) s += l[q] * v[part + 4 * q];
    s += __shfl_xor(s, 1, 64);
    s += __shfl_xor(s, 2, 64);
    return s;
}

__global__ __launch_bounds__(256) void k_backsub_flow(const DenseDesc *__restrict__ desc, DenseParam *__restrict__ prm,
                                                     const double *__restrict__ work, double *__restrict__ x,
                                                     const int64_t *__restrict__ x_off,
                                                     const BsTask *__restrict__ tasks, int32_t n_tasks,
                                                     int *__restrict__ flags, const int64_t *__restrict__ bo,
                                                     int *__restrict__ queue, int *__restrict__ gab_, int limit) {
    __shared__ double xs[2][TB], ys[2][TB];
    __shared__ int s_task;
    __shared__ int s_val;
    const int t = threadIdx.x, o = t >> 2, part = t & 3;
    glb_i32 *gab = (glb_i32 *)gab_;
    for (;;) {
        __syncthreads();   // the previous task's shared values are no longer read
        if (t == 0) s_task = atomicAdd(queue, 1);
        __syncthreads();
        const int ti = s_task;
        if (ti >= n_tasks) return;
        const BsTask tk = tasks[ti];
        const int m = tk.m;
        const DenseDesc d = desc[m];
        if (!prm[m].active || __hip_atomic_load(&prm[m].info, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) continue;
        const int T = (d.n + TB - 1) / TB;
        glb_i32 *fl = (glb_i32 *)(flags + bo[m]);
        glb_i32 *ab = fl + T;
        const int hi = T - 1 - 2 * tk.p, lo = hi - 1;   // lo < 0: none
        const int nh = min(TB, d.n - TB * hi);          // only the last block row can be partial
        const int64_t n = d.n;
        const double *A = work + d.a_off;
        const int64_t xo = x_off[m];
        double lih[16], lil[16], lc[16];
#pragma unroll
        for (int q = 0; q < 16; q++) {
            const int r = part + 4 * q;
            lih[q] = work[d.linv_off + (int64_t)hi * TB * TB + r * TB + o];
            lil[q] = lo >= 0 ? work[d.linv_off + (int64_t)lo * TB * TB + r * TB + o] : 0.0;
            lc[q] = (lo >= 0 && r < nh) ? A[((int64_t)TB * hi + r) * n + (int64_t)TB * lo + o] : 0.0;
        }
        double yh = o < nh ? work[d.v_off + (int64_t)TB * hi + o] : 0.0;
        double yl = lo >= 0 ? work[d.v_off + (int64_t)TB * lo + o] : 0.0;
        bool ok = true;
        for (int pp = 0; pp < tk.p; pp++) {
            const int k1 = T - 1 - 2 * pp, k2 = k1 - 1;   // k2 > hi
            const int n1 = min(TB, d.n - TB * k1);
            double t1h[16], t2h[16], t1l[16], t2l[16];
#pragma unroll
            for (int q = 0; q < 16; q++) {
                const int r = part + 4 * q;
                const int64_t r1 = ((int64_t)TB * k1 + r) * n, r2 = ((int64_t)TB * k2 + r) * n;
                t1h[q] = r < n1 ? A[r1 + (int64_t)TB * hi + o] : 0.0;
                t2h[q] = A[r2 + (int64_t)TB * hi + o];
                t1l[q] = (lo >= 0 && r < n1) ? A[r1 + (int64_t)TB * lo + o] : 0.0;
                t2l[q] = lo >= 0 ? A[r2 + (int64_t)TB * lo + o] : 0.0;
            }
            if (!flow_wait(fl + pp, ab, gab, limit, (lds_i32 *)&s_val)) {
                ok = false;
                break;
            }
            if (t < TB) {
                xs[0][t] = t < n1 ? x[xo + (int64_t)TB * k1 + t] : 0.0;
                xs[1][t] = x[xo + (int64_t)TB * k2 + t];
            }
            __syncthreads();
            yh -= bs_dot16(t1h, xs[0], part);
            yh -= bs_dot16(t2h, xs[1], part);
            yl -= bs_dot16(t1l, xs[0], part);
            yl -= bs_dot16(t2l, xs[1], part);
        }
        if (!ok) {
            if (t == 0) {
                flag_set(ab, __ATOMIC_RELAXED);
                __hip_atomic_store(&prm[m].info, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            continue;
        }
        if (part == 0) ys[0][o] = yh;
        __syncthreads();
        const double xh = bs_dot16(lih, ys[0], part);
        if (part == 0) xs[0][o] = xh;
        __syncthreads();
        double xl = 0.0;
        if (lo >= 0) {
            yl -= bs_dot16(lc, xs[0], part);
            if (part == 0) ys[1][o] = yl;
            __syncthreads();
            xl = bs_dot16(lil, ys[1], part);
        }
        if (part == 0) {
            if (o < nh) x[xo + (int64_t)TB * hi + o] = xh;
            if (lo >= 0) x[xo + (int64_t)TB * lo + o] = xl;
        }
        flow_publish(fl + tk.p);
    }
}

// Back-substitution tasks of one matrix with T block rows (the standalone solve).
__global__ void k_bs_tasks_one(int32_t T, BsTask *__restrict__ tasks) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < (T + 1) / 2) tasks[p] = BsTask{0, p};
}

__global__ void k_fill_i32(int64_t n, int *__restrict__ p, int v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static int64_t flow_task_count(int64_t T) { return 1 + (T >= 3 ? (T - 2) * (T - 3) / 2 + 2 * (T - 2) : 0); }

// ---------------------------------------------------------------- LM glue
// Per-window damping parameters from the LM state and the dense diagonal.
// Gradient norm of every window with fresh derivatives, formed exactly as
// k_dense_params forms it (same partial sums and tree): for a decision that
// must be taken before the dense matrix is assembled, and for the report at
// the end of a run (tol_g > 0: the same convergence test as k_dense_params).
__global__ __launch_bounds__(256) void k_dense_gnorm(int32_t W, const DenseDesc *__restrict__ desc,
                                                     LMState *__restrict__ lm, const double *__restrict__ g,
                                                     double tol_g) {
    __shared__ double rs[256];
    const int w = blockIdx.x;
    if (w >= W) return;
    LMState &st = lm[w];
    if (st.done || !st.need_eval) return;
    const DenseDesc d = desc[w];
    double s = 0.0;
    for (int i = threadIdx.x; i < d.n; i += 256) {
        const double gi = g[6LL * d.pose0 + i];
        s = fma(gi, gi, s);
    }
    rs[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) rs[threadIdx.x] += rs[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        st.gnorm = sqrt(rs[0]);
        if (tol_g > 0.0 && st.gnorm < tol_g) {
            st.done = 1;
            st.accepted = 0;
        }
    }
}

__global__ __launch_bounds__(256) void k_dense_params(int32_t W, const DenseDesc *__restrict__ desc,
                                                      const double *__restrict__ H, const int64_t *__restrict__ h_off,
                                                      LMState *__restrict__ lm, DenseParam *__restrict__ prm,
                                                      double tol_g, const double *__restrict__ g) {
    __shared__ double rm[256], rs[256];
    const int w = blockIdx.x;
    if (w >= W) return;
    LMState &st = lm[w];
    const DenseDesc d = desc[w];
    if (st.done) {
        if (threadIdx.x == 0) prm[w].active = 0;
        return;
    }
    const bool fresh = st.need_eval;
    double mx = 0.0, s = 0.0;
    if (fresh) {
        const double *Hm = H + h_off[w];
        for (int i = threadIdx.x; i < d.n; i += 256) {
            mx = fmax(mx, Hm[(int64_t)i * d.n + i]);
            const double gi = g[6LL * d.pose0 + i];
            s = fma(gi, gi, s);
        }
    }
    rm[threadIdx.x] = mx;
    rs[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            rm[threadIdx.x] = fmax(rm[threadIdx.x], rm[threadIdx.x + o]);
            rs[threadIdx.x] += rs[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (fresh) {
            st.maxdiag = rm[0];
            st.gnorm = sqrt(rs[0]);
            st.need_eval = 0;
            if (tol_g > 0.0 && st.gnorm < tol_g) {
                st.done = 1;
                st.accepted = 0;
            }
        }
        DenseParam p;
        p.mu = st.mu;
        p.floor_ = 1e-12 * st.maxdiag;
        p.active = st.done ? 0 : 1;
        p.info = 0;
        prm[w] = p;
    }
}

// (H dx) per row, one wavefront per row; then per scan: q_j, trial pose, info.
__global__ __launch_bounds__(256) void k_dense_hdx(int32_t W, const DenseDesc *__restrict__ desc,
                                                   const DenseParam *__restrict__ prm, const double *__restrict__ H,
                                                   const int64_t *__restrict__ h_off, const double *__restrict__ dx,
                                                   double *__restrict__ hdx) {
    const int m = blockIdx.y;
    const DenseDesc d = desc[m];
    if (!prm[m].active) return;
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (row >= d.n) return;
    const double *Hr = H + h_off[m] + row * d.n;
    const double *xv = dx + 6LL * d.pose0;
    double s = 0.0;
    for (int64_t c = lane; c < d.n; c += 64) s = fma(Hr[c], xv[c], s);
    s = wave_sum(s);
    if (lane == 0) hdx[6LL * d.pose0 + row] = s;
}

__global__ void k_dense_finish(int32_t n_poses, const int32_t *__restrict__ pose_window,
                               const int32_t *__restrict__ win_pose_ptr, const DenseParam *__restrict__ prm,
                               const double *__restrict__ g, const double *__restrict__ hdx,
                               const double *__restrict__ poses, double *__restrict__ dx,
                               double *__restrict__ pose_q, int32_t *__restrict__ pose_info,
                               double *__restrict__ poses_trial) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_poses) return;
    const int w = pose_window[j];
    const DenseParam p = prm[w];
    if (!p.active) return;
    double *xj = dx + 6LL * j;
    if (p.info) {
#pragma unroll
        for (int k = 0; k < 6; k++) xj[k] = 0.0;
        pose_q[j] = 0.0;
        pose_info[j] = (j == win_pose_ptr[w]) ? p.info : 0;
    } else {
        double gdx = 0.0, dhd = 0.0;
#pragma unroll
        for (int k = 0; k < 6; k++) {
            gdx += g[6LL * j + k] * xj[k];
            dhd += xj[k] * hdx[6LL * j + k];
        }
        pose_q[j] = -(gdx + 0.5 * dhd);
        pose_info[j] = 0;
    }
    pose_plus(poses + 12LL * j, xj, poses_trial + 12LL * j);
}

// Zero the dense matrices of windows whose derivatives are being re-evaluated.
__global__ void k_dense_zero_stale(int32_t W, const DenseDesc *__restrict__ desc, const int64_t *__restrict__ h_off,
                                   const LMState *__restrict__ lm, double *__restrict__ dense) {
    for (int w = 0; w < W; w++) {
        const LMState &st = lm[w];
        if (st.done || !st.need_eval) continue;
        const int64_t a = h_off[w], b = h_off[w + 1];
        for (int64_t i = a + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < b;
             i += (int64_t)gridDim.x * blockDim.x)
            dense[i] = 0.0;
    }
}

// ---------------------------------------------------------------- host side
static inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// Compute units of the current device.
static int cu_count() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    return cus;
}

// Polls before a wait of the dataflow factorization gives up: FLOW_SPIN, or
// the environment's BA_FLOW_SPIN (a negative value gives up at once, which
// the tests use to exercise the abort path).
static int flow_spin_limit() {
    const char *e = getenv("BA_FLOW_SPIN");
    return e ? atoi(e) : FLOW_SPIN;
}

// Dataflow factorization and forward substitution (k_chol_flow): flags,
// tickets and the abort flag cleared by a kernel (no memset node in a
// captured graph), then one persistent launch per group of matrices.
struct DenseState {
    DevArena mem;
    bool ready = false;
    // pairs
    int32_t n_seg = 0;
    PairSeg *segs = nullptr;
    int32_t *pa = nullptr, *pb = nullptr;
    double *h = nullptr;
    // exact form: voxel ranges of the voxel-major clusters, 3 vectors per cluster
    int32_t n_vx = 0;
    int64_t *vptr = nullptr;
    double *ev = nullptr;
    // matrices
    DenseDesc *desc = nullptr;
    DenseParam *prm = nullptr;
    int64_t *h_off = nullptr;    // offsets of each window's undamped H in P->dense
    int64_t *x_off = nullptr;    // offsets of each window's solution in P->dx
    double *work = nullptr;
    double *hdx = nullptr;
    int32_t max_n = 0;
    // dataflow factorization (every matrix at most FLOW_MAX_N): task list,
    // per-matrix flags at flow_fo[m], then one queue ticket per launch and the
    // abort flag; launch q takes tasks [flow_first[q], + flow_count[q])
    FlowTask *flow_tasks = nullptr;
    int *flow_flags = nullptr;
    int64_t *flow_fo = nullptr;
    int64_t flow_ints = 0;
    std::vector<int32_t> flow_first, flow_count;
    std::vector<int32_t> flow_mats;   // matrices (walkers) of each launch
    std::vector<int64_t> flow_work;   // sum of T^2 over the launch's matrices (sets its helper count)
    // dataflow back substitution: its flags follow the factorization's in
    // flow_flags (per matrix T + 1 at bs_bo[m], then a queue ticket and an
    // abort flag at bs_ticket, bs_ticket + 1); bs_ints counts them all
    BsTask *bs_tasks = nullptr;
    int32_t bs_count = 0;
    int64_t *bs_bo = nullptr;
    int64_t bs_ticket = 0, bs_ints = 0;
};

static DenseState *dense_state(Problem *P) { return (DenseState *)P->dense_state; }

void dense_release(Problem *P) {
    delete dense_state(P);
    P->dense_state = nullptr;
}

static int64_t linv_doubles(int64_t n) { return ((n + TB - 1) / TB) * (int64_t)TB * TB; }

double *dense_hvec(Problem *P) {
    DenseState *D = (DenseState *)P->dense_state;
    return D ? D->h : nullptr;
}

// ---------------------------------------------------------------- pair plan
// Every (voxel, i <= j) pair of a voxel's clusters, in the order of the voxels
// and, within one, cluster i outer and j inner, keyed by their scans
// (j_i << bits_b | j_j); a voxel's clusters are in scan order, so j_i <= j_j.
// A stable sort by the key then lists the pairs by (j_i, j_j) with ties in
// this order.
__global__ void k_pair_emit(int32_t n_vx, const int64_t *__restrict__ vptr, const int64_t *__restrict__ poff,
                            const int32_t *__restrict__ cscan, int bits_b, uint64_t *__restrict__ keys,
                            uint32_t *__restrict__ vals, int32_t *__restrict__ ea, int32_t *__restrict__ eb) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n_vx) return;
    const int64_t a = vptr[v], b = vptr[v + 1];
    int64_t q = poff[v];
    for (int64_t i = a; i < b; i++) {
        const uint64_t ki = (uint64_t)cscan[i] << bits_b;
        for (int64_t j = i; j < b; j++, q++) {
            keys[q] = ki | (uint64_t)cscan[j];
            vals[q] = (uint32_t)q;
            ea[q] = (int32_t)i;
            eb[q] = (int32_t)j;
        }
    }
}

__global__ void k_inv_perm(int64_t C, const int32_t *__restrict__ perm, int32_t *__restrict__ inv) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < C) inv[perm[q]] = (int32_t)q;
}

// Sorted pairs: their clusters in the order h is kept in (qc maps a
// voxel-major cluster to it; null: voxel-major) and a 1 at each new key.
__global__ void k_pair_out(int64_t E, const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals,
                           const int32_t *__restrict__ ea, const int32_t *__restrict__ eb,
                           const int32_t *__restrict__ qc, int32_t *__restrict__ spa, int32_t *__restrict__ spb,
                           int64_t *__restrict__ head) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= E) return;
    const uint32_t o = vals[r];
    const int32_t a = ea[o], b = eb[o];
    spa[r] = qc ? qc[a] : a;
    spb[r] = qc ? qc[b] : b;
    head[r] = (r == 0 || keys[r] != keys[r - 1]) ? 1 : 0;
}

// One segment per key: its start (sidx = exclusive scan of the key heads),
// then its length from the next segment's start.
__global__ void k_seg_emit(int64_t E, const uint64_t *__restrict__ keys, const int64_t *__restrict__ sidx,
                           int bits_b, PairSeg *__restrict__ segs) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= E || !(r == 0 || keys[r] != keys[r - 1])) return;
    PairSeg sg;
    sg.start = r;
    sg.count = 0;
    sg.ja = (int32_t)(keys[r] >> bits_b);
    sg.jb = (int32_t)(keys[r] & ((1ULL << bits_b) - 1));
    sg.pad = 0;
    segs[sidx[r]] = sg;
}

__global__ void k_seg_count(int64_t n_seg, int64_t E, PairSeg *__restrict__ segs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_seg) segs[i].count = (int32_t)((i + 1 < n_seg ? segs[i + 1].start : E) - segs[i].start);
}

int64_t dense_device_bytes(const Problem *P) {
    const DenseState *D = (const DenseState *)P->dense_state;
    return D ? (int64_t)D->mem.bytes : 0;
}

ba_status dense_prepare(Problem *P) {
    if (P->dense_state) return BA_OK;
    hipStream_t s = 0;
    DenseState *D = new DenseState();
    P->dense_state = D;
    const int64_t C = P->n_clusters;
    const int32_t W = P->n_windows;
    // voxel runs of the voxel-major clusters and their pair counts (host),
    // then the pairs themselves, sorted by their scan pair on the device
    std::vector<int32_t> cvox(C);
    BA_HIP(hipMemcpy(cvox.data(), P->c_vox, sizeof(int32_t) * C, hipMemcpyDeviceToHost));
    std::vector<int64_t> vptr, poff;
    vptr.reserve((size_t)C / 2 + 2);
    poff.reserve((size_t)C / 2 + 2);
    int64_t E = 0;
    for (int64_t a = 0; a < C;) {
        int64_t b = a;
        while (b < C && cvox[b] == cvox[a]) b++;
        vptr.push_back(a);
        poff.push_back(E);
        E += (b - a) * (b - a + 1) / 2;
        a = b;
    }
    vptr.push_back(C);
    poff.push_back(E);
    D->n_vx = (int32_t)vptr.size() - 1;
    if (E >= (int64_t)UINT32_MAX) {
        set_error("%lld cluster pairs exceed the pair plan's 2^32 limit", (long long)E);
        return BA_E_UNSUPPORTED;
    }
    BA_TRY(D->mem.alloc(&D->vptr, (int64_t)vptr.size()));
    BA_HIP(hipMemcpy(D->vptr, vptr.data(), sizeof(int64_t) * vptr.size(), hipMemcpyHostToDevice));
    BA_TRY(D->mem.alloc(&D->pa, std::max<int64_t>(E, 1)));
    BA_TRY(D->mem.alloc(&D->pb, std::max<int64_t>(E, 1)));
    BA_TRY(D->mem.alloc(&D->h, 6 * std::max<int64_t>(C, 1)));
    D->n_seg = 0;
    if (E > 0) {
        const int32_t NP = P->n_poses;
        int bits_b = 1;
        while (bits_b < 31 && (int64_t(1) << bits_b) < NP) bits_b++;
        DevArena tmp;
        int64_t *d_poff, *head, *d_total;
        uint64_t *keys;
        uint32_t *vals;
        int32_t *ea, *eb, *qc = nullptr;
        char *ws;
        const size_t ws_bytes = std::max(radix_sort_workspace_bytes(E), scan_workspace_bytes(E));
        BA_TRY(tmp.alloc(&d_poff, (int64_t)poff.size()));
        BA_TRY(tmp.alloc(&keys, E));
        BA_TRY(tmp.alloc(&vals, E));
        BA_TRY(tmp.alloc(&ea, E));
        BA_TRY(tmp.alloc(&eb, E));
        BA_TRY(tmp.alloc(&head, E));
        BA_TRY(tmp.alloc(&d_total, 1));
        BA_TRY(tmp.alloc(&ws, (int64_t)ws_bytes));
        BA_HIP(hipMemcpy(d_poff, poff.data(), sizeof(int64_t) * poff.size(), hipMemcpyHostToDevice));
        hipLaunchKernelGGL(k_pair_emit, dim3(nblk(D->n_vx)), dim3(256), 0, s, D->n_vx, D->vptr, d_poff, P->c_scan,
                           bits_b, keys, vals, ea, eb);
        BA_HIP(radix_sort_pairs(keys, vals, E, 2 * bits_b, ws, s));
        // the precision form keeps h in the order of its derivative pass's
        // cluster copy: the pair lists then index that order
        if (P->prec == BA_PREC_F32) {
            BA_TRY(tmp.alloc(&qc, C));
            hipLaunchKernelGGL(k_inv_perm, dim3(nblk(C)), dim3(256), 0, s, C, P->p_cidx, qc);
        }
        hipLaunchKernelGGL(k_pair_out, dim3(nblk(E)), dim3(256), 0, s, E, keys, vals, ea, eb, qc, D->pa, D->pb,
                           head);
        BA_HIP(exclusive_scan_i64(head, head, E, d_total, ws, s));
        int64_t n_seg = 0;
        BA_HIP(hipMemcpy(&n_seg, d_total, sizeof(int64_t), hipMemcpyDeviceToHost));
        D->n_seg = (int32_t)n_seg;
        BA_TRY(D->mem.alloc(&D->segs, std::max<int64_t>(n_seg, 1)));
        hipLaunchKernelGGL(k_seg_emit, dim3(nblk(E)), dim3(256), 0, s, E, keys, head, bits_b, D->segs);
        hipLaunchKernelGGL(k_seg_count, dim3(nblk(n_seg)), dim3(256), 0, s, n_seg, E, D->segs);
        BA_HIP(hipStreamSynchronize(s));   // before the temporaries go
    } else {
        BA_TRY(D->mem.alloc(&D->segs, 1));
    }
    // per-window dense matrices
    std::vector<DenseDesc> desc(W);
    std::vector<int64_t> hoff(W + 1), xoff(W);
    int64_t a_tot = 0, l_tot = 0, v_tot = 0, h_tot = 0;
    for (int32_t w = 0; w < W; w++) {
        const int32_t p0 = P->h_win_pose_ptr[w], p1 = P->h_win_pose_ptr[w + 1];
        const int64_t n = 6LL * (p1 - p0);
        desc[w].a_off = a_tot;
        desc[w].linv_off = l_tot;
        desc[w].v_off = v_tot;
        desc[w].n = (int32_t)n;
        desc[w].pose0 = p0;
        hoff[w] = h_tot;
        xoff[w] = 6LL * p0;
        a_tot += n * n;
        l_tot += linv_doubles(n);
        v_tot += n;
        h_tot += n * n;
        D->max_n = std::max<int32_t>(D->max_n, (int32_t)n);
    }
    hoff[W] = h_tot;
    BA_TRY(D->mem.alloc(&D->desc, W));
    BA_TRY(D->mem.alloc(&D->prm, W));
    BA_TRY(D->mem.alloc(&D->h_off, W + 1));
    BA_TRY(D->mem.alloc(&D->x_off, W));
    BA_TRY(D->mem.alloc(&D->work, a_tot + l_tot + v_tot));
    BA_TRY(D->mem.alloc(&D->hdx, 6LL * P->n_poses));
    BA_TRY(D->mem.alloc(&P->dense, std::max<int64_t>(h_tot, 1)));
    P->dense_total = h_tot;
    for (int32_t w = 0; w < W; w++) {
        desc[w].linv_off += a_tot;
        desc[w].v_off += a_tot + l_tot;
    }
    BA_HIP(hipMemcpy(D->desc, desc.data(), sizeof(DenseDesc) * W, hipMemcpyHostToDevice));
    BA_HIP(hipMemcpy(D->h_off, hoff.data(), sizeof(int64_t) * (W + 1), hipMemcpyHostToDevice));
    BA_HIP(hipMemcpy(D->x_off, xoff.data(), sizeof(int64_t) * W, hipMemcpyHostToDevice));
    BA_HIP(hipMemset(P->dense, 0, sizeof(double) * std::max<int64_t>(h_tot, 1)));
    if (D->max_n <= FLOW_MAX_N) {
        // walkers of up to FLOW_MAX_MATS matrices per launch, then their
        // tasks by column
        std::vector<FlowTask> tasks;
        std::vector<int64_t> fo(W);
        int64_t ints = 0;
        for (int32_t w = 0; w < W; w++) {
            fo[w] = ints;
            ints += flow_flag_ints((desc[w].n + TB - 1) / TB);
        }
        // walkers of a launch hold at most half of the compute units, so that
        // every launch keeps workgroups for its helpers
        const int32_t per_launch = std::max(1, std::min(FLOW_MAX_MATS, cu_count() / 2));
        for (int32_t m0 = 0; m0 < W; m0 += per_launch) {
            const int32_t m1 = std::min<int32_t>(W, m0 + per_launch);
            D->flow_first.push_back((int32_t)tasks.size());
            int32_t maxT = 0;
            for (int32_t m = m0; m < m1; m++) {
                tasks.push_back(FlowTask{m, FLOW_WALK, 0, 0});
                maxT = std::max<int32_t>(maxT, (desc[m].n + TB - 1) / TB);
            }
            for (int32_t c = 0; c < maxT; c++)
                for (int32_t m = m0; m < m1; m++) {
                    const int32_t T = (desc[m].n + TB - 1) / TB;
                    for (int32_t i = c + 3; i < T; i++) tasks.push_back(FlowTask{m, FLOW_TILE, i, c});
                    if (c + 2 <= T - 1) {
                        tasks.push_back(FlowTask{m, FLOW_PDIAG, c + 2, c});
                        tasks.push_back(FlowTask{m, FLOW_POFF, c + 2, c});
                    }
                }
            D->flow_count.push_back((int32_t)tasks.size() - D->flow_first.back());
            int64_t work = 0;
            for (int32_t m = m0; m < m1; m++) {
                const int64_t T = (desc[m].n + TB - 1) / TB;
                work += T * T;
            }
            D->flow_mats.push_back(m1 - m0);
            D->flow_work.push_back(work);
        }
        D->flow_ints = ints;
        // back substitution: tasks p-major over the matrices, flags after the
        // factorization's tickets and abort flag
        std::vector<BsTask> bs;
        std::vector<int64_t> bo(W);
        int64_t bints = ints + (int64_t)D->flow_first.size() + 1;
        const int64_t bs_base = bints;
        int32_t maxP = 0;
        for (int32_t w = 0; w < W; w++) {
            const int32_t T = (desc[w].n + TB - 1) / TB;
            bo[w] = bints;
            bints += T + 1;
            maxP = std::max(maxP, (T + 1) / 2);
        }
        for (int32_t p = 0; p < maxP; p++)
            for (int32_t w = 0; w < W; w++)
                if (p < ((desc[w].n + TB - 1) / TB + 1) / 2) bs.push_back(BsTask{w, p});
        D->bs_ticket = bints;
        D->bs_ints = bints + 2 - bs_base;
        D->bs_count = (int32_t)bs.size();
        BA_TRY(D->mem.alloc(&D->flow_tasks, (int64_t)tasks.size()));
        BA_TRY(D->mem.alloc(&D->flow_flags, bints + 2));
        BA_TRY(D->mem.alloc(&D->flow_fo, W));
        BA_TRY(D->mem.alloc(&D->bs_tasks, std::max<int64_t>(D->bs_count, 1)));
        BA_TRY(D->mem.alloc(&D->bs_bo, W));
        BA_HIP(hipMemcpy(D->flow_tasks, tasks.data(), sizeof(FlowTask) * tasks.size(), hipMemcpyHostToDevice));
        BA_HIP(hipMemcpy(D->flow_fo, fo.data(), sizeof(int64_t) * W, hipMemcpyHostToDevice));
        if (!bs.empty())
            BA_HIP(hipMemcpy(D->bs_tasks, bs.data(), sizeof(BsTask) * bs.size(), hipMemcpyHostToDevice));
        BA_HIP(hipMemcpy(D->bs_bo, bo.data(), sizeof(int64_t) * W, hipMemcpyHostToDevice));
    }
    D->ready = true;
    return BA_OK;
}

// Coupled Hessian at `poses` into hess_out (one window, standalone) or into
// the problem's per-window dense buffers (LM).
ba_status dense_assemble(Problem *P, const double *poses, double *hess_out, bool use_lm, hipStream_t s) {
    BA_TRY(dense_prepare(P));
    DenseState *D = dense_state(P);
    double *dst = hess_out ? hess_out : P->dense;
    const LMState *lm = use_lm ? P->lm : nullptr;
    const int64_t C = P->n_clusters;
    // the precision form takes h from the derivative pass (the same FP32
    // clusters as the per-pose blocks, so the pair blocks cancel the diagonal
    // blocks exactly along the translation gauge)
    if (P->prec != BA_PREC_F32)
        hipLaunchKernelGGL(k_hvec, dim3(nblk(C)), dim3(256), 0, s, C, P->c_N, P->c_mu, P->c_scan, P->c_slot, poses,
                           P->vstate, (int64_t)P->n_groups * 64, P->pose_window, lm, D->h);
    // windows whose derivatives are stale are rebuilt whole; the others keep their matrix
    if (!use_lm) {
        const int64_t tot = P->dense_total;
        hipLaunchKernelGGL(k_fill, dim3(nblk(tot)), dim3(256), 0, s, tot, dst, 0.0);
    } else {
        hipLaunchKernelGGL(k_dense_zero_stale, dim3(2048), dim3(256), 0, s, P->n_windows, D->desc, D->h_off, lm,
                           dst);
    }
    if (D->n_seg)
        hipLaunchKernelGGL(k_pairs, dim3(nblk((int64_t)D->n_seg * 64)), dim3(256), 0, s, D->n_seg, D->segs, D->pa,
                           D->pb, D->h, P->H, P->pose_window, P->win_pose_ptr, D->h_off, lm, dst);
    BA_HIP(hipGetLastError());
    return BA_OK;
}

// Exact Hessian at `poses` (FP64 problems; the per-pose blocks P->H must hold
// the MM Hessian at the same poses) into hess_out, or with the LM the
// per-window dense buffers with the exact terms for windows whose gradient
// norm is below exact_below.
ba_status dense_assemble_exact(Problem *P, const double *poses, double *hess_out, bool use_lm, double exact_below,
                               hipStream_t s) {
    BA_TRY(dense_prepare(P));
    DenseState *D = dense_state(P);
    if (P->prec != BA_PREC_F64) {
        set_error("the exact Hessian is built for FP64 problems only");
        return BA_E_UNSUPPORTED;
    }
    if (!D->ev) BA_TRY(D->mem.alloc(&D->ev, 18 * std::max<int64_t>(P->n_clusters, 1)));
    double *dst = hess_out ? hess_out : P->dense;
    const LMState *lm = use_lm ? P->lm : nullptr;
    hipLaunchKernelGGL(k_exact_vecs, dim3(nblk(D->n_vx)), dim3(256), 0, s, D->n_vx, D->vptr, P->c_N, P->c_mu,
                       P->c_S, P->c_scan, poses, D->ev);
    if (!use_lm) {
        const int64_t tot = P->dense_total;
        hipLaunchKernelGGL(k_fill, dim3(nblk(tot)), dim3(256), 0, s, tot, dst, 0.0);
    } else {
        hipLaunchKernelGGL(k_dense_zero_stale, dim3(2048), dim3(256), 0, s, P->n_windows, D->desc, D->h_off, lm,
                           dst);
    }
    if (D->n_seg)
        hipLaunchKernelGGL(k_pairs_x, dim3(nblk((int64_t)D->n_seg * 64)), dim3(256), 0, s, D->n_seg, D->segs, D->pa,
                           D->pb, D->ev, P->H, P->pose_window, P->win_pose_ptr, D->h_off, lm, exact_below, dst);
    BA_HIP(hipGetLastError());
    return BA_OK;
}

static void launch_flow_factor(DenseState *D, const double *H, const int64_t *h_off, const double *g,
                               hipStream_t s) {
    const int nl = (int)D->flow_first.size();
    const int64_t nint = D->flow_ints + nl + 1 + D->bs_ints;   // the back substitution's flags follow
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)std::min<int64_t>(nblk(nint), 1024)), dim3(256), 0, s, nint,
                       D->flow_flags, 0);
    const int limit = flow_spin_limit();
    // one workgroup per compute unit (the walker's factor and the partial
    // tasks' accumulators need more than half of the register file): the
    // walkers plus helpers in proportion to the tiles, so that the early
    // steps of a large matrix have the whole device while small problems
    // solved side by side (concurrent streams) leave room for each other
    const int cus = cu_count();
    for (int q = 0; q < nl; q++) {
        const int64_t helpers = std::max<int64_t>(32, D->flow_work[q] / 8);
        const int grid = (int)std::min<int64_t>({(int64_t)D->flow_count[q], (int64_t)cus, D->flow_mats[q] + helpers});
        ProfScope prof("k_chol_flow", s);
        hipLaunchKernelGGL(k_chol_flow, dim3((unsigned)grid), dim3(256), 0, s, D->desc,
                           D->prm, H, h_off, g, D->work, D->flow_tasks + D->flow_first[q], D->flow_count[q],
                           D->flow_flags, D->flow_fo, D->flow_flags + D->flow_ints + q,
                           D->flow_flags + D->flow_ints + nl, limit);
    }
}

// Blocked right-looking factorization, one launch per step: panels of PANEL
// 64-wide steps; a step updates the rest of its panel, each panel then the
// trailing matrix with K = the panel's width (one read and write of the
// trailing matrix per panel instead of per step).
static void launch_blocked_factor(DenseState *D, int32_t nmat, int nsteps, hipStream_t s) {
    constexpr int PANEL = 4;
    for (int p = 0; p < nsteps; p += PANEL) {
        const int pe = std::min(p + PANEL, nsteps);
        for (int st = p; st < pe; st++) {
            {
                ProfScope prof("k_potf2", s);
                hipLaunchKernelGGL(k_potf2, dim3(1, nmat), dim3(256), 0, s, D->desc, D->prm, D->work, st);
            }
            const int64_t below = nsteps - st - 1;
            if (below > 0) {
                {
                    ProfScope prof("k_trsm", s);
                    hipLaunchKernelGGL(k_trsm, dim3((unsigned)below, nmat), dim3(256), 0, s, D->desc, D->prm,
                                       D->work, st);
                }
                const int64_t cols = pe - st - 1;   // tile columns left in the panel
                if (cols > 0) {
                    const int64_t tiles = cols * below - cols * (cols - 1) / 2;
                    ProfScope prof("k_syrk", s);
                    hipLaunchKernelGGL(k_syrk, dim3((unsigned)tiles, nmat), dim3(256), 0, s, D->desc, D->prm,
                                       D->work, st, TB, st + 1, pe);
                }
            }
        }
        const int64_t rest = nsteps - pe;
        if (rest > 0) {
            ProfScope prof("k_syrk", s);
            hipLaunchKernelGGL(k_syrk, dim3((unsigned)(rest * (rest + 1) / 2), nmat), dim3(256), 0, s, D->desc,
                               D->prm, D->work, p, TB * (pe - p), pe, nsteps);
        }
    }
}

static void launch_factor_solve(DenseState *D, int32_t nmat, int32_t max_n, const double *H, const int64_t *h_off,
                                const double *g, double *x, const int64_t *x_off, hipStream_t s) {
    const int nsteps = (max_n + TB - 1) / TB;
    const int64_t nn = (int64_t)max_n * max_n;
    if (D->flow_tasks && max_n <= FLOW_MAX_N) {
        launch_flow_factor(D, H, h_off, g, s);   // reads H and g directly (and clears both kernels' flags)
        // back substitution in one launch: tasks of a matrix mostly wait on
        // each other, so a few per compute unit
        const int grid = (int)std::min<int64_t>(D->bs_count, 2LL * cu_count());
        if (grid > 0) {
            ProfScope prof("k_backsub_flow", s);
            hipLaunchKernelGGL(k_backsub_flow, dim3((unsigned)grid), dim3(256), 0, s, D->desc, D->prm, D->work, x,
                               x_off, D->bs_tasks, D->bs_count, D->flow_flags, D->bs_bo,
                               D->flow_flags + D->bs_ticket, D->flow_flags + D->bs_ticket + 1, flow_spin_limit());
        }
        return;
    } else {
        hipLaunchKernelGGL(k_damp_copy, dim3((unsigned)std::min<int64_t>(nblk(nn), 4096), nmat), dim3(256), 0, s,
                           D->desc, D->prm, H, h_off, g, D->work);
        launch_blocked_factor(D, nmat, nsteps, s);
    }
    // launch-per-step path: backward substitution two block rows per launch
    // (every workgroup loads the rows' inverse and cross tiles: with three rows
    // its 145 loads per thread need three rounds of outstanding loads, 15 us a
    // launch)
    constexpr int BR = 2;
    for (int st = nsteps - 1; st >= 0; st -= BR) {
        ProfScope prof("k_backsub_rows", s);
        hipLaunchKernelGGL(k_backsub_rows<BR>, dim3((unsigned)std::max(st - BR + 1, 1), nmat), dim3(256), 0, s,
                           D->desc, D->prm, D->work, x, x_off, st);
    }
}

void launch_dense_gnorm(Problem *P, hipStream_t s, double tol_g) {
    DenseState *D = dense_state(P);
    hipLaunchKernelGGL(k_dense_gnorm, dim3(P->n_windows), dim3(256), 0, s, P->n_windows, D->desc, P->lm, P->g,
                       tol_g);
}

ba_status dense_lm_step(Problem *P, const double *poses, double tol_g, hipStream_t s) {
    DenseState *D = dense_state(P);
    const int32_t W = P->n_windows;
    hipLaunchKernelGGL(k_dense_params, dim3(W), dim3(256), 0, s, W, D->desc, P->dense, D->h_off, P->lm, D->prm, tol_g,
                       P->g);
    launch_factor_solve(D, W, D->max_n, P->dense, D->h_off, P->g, P->dx, D->x_off, s);
    hipLaunchKernelGGL(k_dense_hdx, dim3(nblk((int64_t)D->max_n * 64), W), dim3(256), 0, s, W, D->desc, D->prm,
                       P->dense, D->h_off, P->dx, D->hdx);
    hipLaunchKernelGGL(k_dense_finish, dim3(nblk(P->n_poses)), dim3(256), 0, s, P->n_poses, P->pose_window,
                       P->win_pose_ptr, D->prm, P->g, D->hdx, poses, P->dx, P->pose_q, P->pose_info,
                       P->poses_trial);
    BA_HIP(hipGetLastError());
    return BA_OK;
}

// ---------------------------------------------------------------- standalone solve
// Workspace of the standalone solve: descriptors, the matrix, the inverse
// blocks and the right-hand side, then (dataflow path) flags, ticket, abort
// flag and task list.
static size_t solve_head_bytes() { return align_up(sizeof(DenseDesc) + sizeof(DenseParam) + 4 * sizeof(int64_t), 256); }
static size_t solve_work_bytes(int64_t n) {
    return align_up(sizeof(double) * (size_t)(n * n + linv_doubles(n) + n), 256);
}
// Flags of the standalone dataflow path: the factorization's, its ticket and
// abort flag, then the back substitution's T + 1, its ticket and abort flag.
static int64_t solve_flag_ints(int64_t T) { return flow_flag_ints(T) + 2 + (T + 1) + 2; }
static size_t solve_flag_bytes(int64_t n) {
    const int64_t T = (n + TB - 1) / TB;
    return n <= FLOW_MAX_N ? align_up(sizeof(int) * (size_t)solve_flag_ints(T), 256) : 0;
}
static size_t solve_task_bytes(int64_t n) {
    const int64_t T = (n + TB - 1) / TB;
    return n <= FLOW_MAX_N ? align_up(sizeof(FlowTask) * (size_t)flow_task_count(T), 256) : 0;
}
size_t dense_solve_workspace(int64_t n) {
    const int64_t T = (n + TB - 1) / TB;
    const size_t bs = n <= FLOW_MAX_N ? sizeof(BsTask) * (size_t)((T + 1) / 2) : 0;
    return solve_head_bytes() + solve_work_bytes(n) + solve_flag_bytes(n) + solve_task_bytes(n) + bs + 256;
}

__global__ void k_solve_setup(int64_t n, const double *__restrict__ H, double mu, DenseDesc *__restrict__ desc,
                              DenseParam *__restrict__ prm, int64_t *__restrict__ offs) {
    __shared__ double rm[256];
    double mx = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) mx = fmax(mx, H[i * n + i]);
    rm[threadIdx.x] = mx;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) rm[threadIdx.x] = fmax(rm[threadIdx.x], rm[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        DenseDesc d;
        d.a_off = 0;
        d.linv_off = n * n;
        d.v_off = n * n + ((n + TB - 1) / TB) * (int64_t)TB * TB;
        d.n = (int32_t)n;
        d.pose0 = 0;
        desc[0] = d;
        DenseParam p;
        p.mu = mu;
        p.floor_ = 1e-12 * rm[0];
        p.active = 1;
        p.info = 0;
        prm[0] = p;
        const int64_t T = (n + TB - 1) / TB;
        offs[0] = 0;  // h_off
        offs[1] = 0;  // x_off
        offs[2] = 0;  // offset of the matrix's factorization flags
        offs[3] = flow_flag_ints(T) + 2;   // offset of its back-substitution flags
    }
}

__global__ void k_solve_final(int64_t n, const DenseParam *__restrict__ prm, double *__restrict__ dx,
                              int32_t *__restrict__ info) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int inf = prm[0].info;
    if (i == 0) *info = inf;
    if (inf && i < n) dx[i] = 0.0;
}

ba_status dense_solve(int64_t n, const double *A, const double *g, double mu, double *dx, int32_t *info, void *ws,
                      size_t ws_bytes, hipStream_t s) {
    char *p = (char *)ws;
    DenseDesc *desc = (DenseDesc *)p;
    DenseParam *prm = (DenseParam *)(p + sizeof(DenseDesc));
    int64_t *offs = (int64_t *)(p + sizeof(DenseDesc) + sizeof(DenseParam));
    double *work = (double *)(p + solve_head_bytes());
    hipLaunchKernelGGL(k_solve_setup, dim3(1), dim3(256), 0, s, n, A, mu, desc, prm, offs);
    DenseState tmp;
    tmp.desc = desc;
    tmp.prm = prm;
    tmp.work = work;
    if (n <= FLOW_MAX_N) {
        const int64_t T = (n + TB - 1) / TB;
        tmp.flow_flags = (int *)(p + solve_head_bytes() + solve_work_bytes(n));
        tmp.flow_tasks = (FlowTask *)(p + solve_head_bytes() + solve_work_bytes(n) + solve_flag_bytes(n));
        tmp.flow_fo = offs + 2;
        tmp.flow_ints = flow_flag_ints(T);
        tmp.flow_first.push_back(0);
        tmp.flow_count.push_back((int32_t)flow_task_count(T));
        tmp.flow_mats.push_back(1);
        tmp.flow_work.push_back(T * T);
        tmp.bs_tasks = (BsTask *)(p + solve_head_bytes() + solve_work_bytes(n) + solve_flag_bytes(n) +
                                  solve_task_bytes(n));
        tmp.bs_count = (int32_t)((T + 1) / 2);
        tmp.bs_bo = offs + 3;
        tmp.bs_ticket = flow_flag_ints(T) + 2 + T + 1;
        tmp.bs_ints = T + 1 + 2;
        hipLaunchKernelGGL(k_flow_tasks_one, dim3(nblk(T)), dim3(256), 0, s, (int32_t)T, tmp.flow_tasks);
        hipLaunchKernelGGL(k_bs_tasks_one, dim3(nblk((T + 1) / 2)), dim3(256), 0, s, (int32_t)T, tmp.bs_tasks);
    }
    launch_factor_solve(&tmp, 1, (int32_t)n, A, offs, g, dx, offs + 1, s);
    hipLaunchKernelGGL(k_solve_final, dim3(nblk(n)), dim3(256), 0, s, n, prm, dx, info);
    BA_HIP(hipGetLastError());
    return BA_OK;
}

}  // namespace ba
