// Problem build: raw points (or raw-sum clusters) -> centred point clusters
// (Eq. 2) -> static plan of the iteration.  Runs once per problem.
//
// Paper Sec. IV-A groups points by (voxel, pose) with sort_by_key and
// reduce_by_key and builds two index mappers, M_v (cluster -> voxel) and M_s
// (voxel-sorted -> pose-sorted order), consumed every iteration (Alg. 2).
// Here the same grouping runs as a stable device radix sort plus one
// wavefront per cluster, and the mappers are materialised once as two
// physical copies of the clusters:
//   * a voxel-major, wave-interleaved copy: voxels of equal cluster count m
//     are packed 64 to a wave group, cluster k of lane l at cbase + 64 k + l,
//     so the residual pass reads fully coalesced with no divergence;
//   * a pose-major copy cut into chunks of one pose, so the derivative pass
//     reduces per pose in registers without scatter or atomics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "ba.h"
#include "ba_device.hpp"
#include "ba_internal.hpp"
#include "ba_host.hpp"

namespace ba {

// ---------------------------------------------------------------- kernels
__global__ void k_validate_points(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                                  const double *__restrict__ z, const int32_t *__restrict__ scan,
                                  const int32_t *__restrict__ voxel, int32_t n_scans, int32_t n_voxels,
                                  int32_t *__restrict__ err) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int bad = 0;
    if (!(isfinite(x[i]) && isfinite(y[i]) && isfinite(z[i]))) bad |= 1;
    if (scan[i] < 0 || scan[i] >= n_scans) bad |= 2;
    if (voxel[i] < 0 || voxel[i] >= n_voxels) bad |= 4;
    if (bad) atomicOr(err, bad);
}

__global__ void k_make_keys(int64_t n, const int32_t *__restrict__ scan, const int32_t *__restrict__ voxel,
                            int32_t n_scans, uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    keys[i] = (uint64_t)voxel[i] * (uint64_t)n_scans + (uint64_t)scan[i];
    vals[i] = (uint32_t)i;
}

__global__ void k_head_flags(int64_t n, const uint64_t *__restrict__ keys, int64_t *__restrict__ flags) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    flags[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

// after an exclusive scan of the head flags: starts[cid] = i for every head
__global__ void k_segment_starts(int64_t n, const uint64_t *__restrict__ keys, const int64_t *__restrict__ excl,
                                 int64_t *__restrict__ starts, int64_t n_seg) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (i == 0 || keys[i] != keys[i - 1]) starts[excl[i]] = i;
    if (i == 0) starts[n_seg] = n;
}

__global__ void k_gather_xyz(int64_t n, const uint32_t *__restrict__ idx, const double *__restrict__ x,
                             const double *__restrict__ y, const double *__restrict__ z, double *__restrict__ xs,
                             double *__restrict__ ys, double *__restrict__ zs) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t j = idx[i];
    xs[i] = x[j];
    ys[i] = y[j];
    zs[i] = z[j];
}

__device__ __forceinline__ double dd_div_int(double hi, double lo, double n) {
    double q = hi / n;
    double r = fma(-q, n, hi) + lo;
    return q + r / n;
}

// One wavefront per cluster: compensated centroid, then centred scatter.
__global__ __launch_bounds__(256) void k_cluster_stats(int64_t C, const int64_t *__restrict__ starts,
                                                       const double *__restrict__ xs, const double *__restrict__ ys,
                                                       const double *__restrict__ zs,
                                                       const uint64_t *__restrict__ skeys, int32_t n_scans,
                                                       double *__restrict__ cN, double *__restrict__ cmu,
                                                       double *__restrict__ cS, int32_t *__restrict__ cvox,
                                                       int32_t *__restrict__ cscan) {
    int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    int lane = threadIdx.x & 63;
    if (c >= C) return;
    int64_t a = starts[c], b = starts[c + 1];
    double hx = 0, lx = 0, hy = 0, ly = 0, hz = 0, lz = 0;
    for (int64_t i = a + lane; i < b; i += 64) {
        dd_add(hx, lx, xs[i]);
        dd_add(hy, ly, ys[i]);
        dd_add(hz, lz, zs[i]);
    }
    wave_dd_sum(hx, lx);
    wave_dd_sum(hy, ly);
    wave_dd_sum(hz, lz);
    double n = (double)(b - a);
    double mx = dd_div_int(hx, lx, n), my = dd_div_int(hy, ly, n), mz = dd_div_int(hz, lz, n);
    double sxx = 0, sxy = 0, sxz = 0, syy = 0, syz = 0, szz = 0;
    for (int64_t i = a + lane; i < b; i += 64) {
        double dx = xs[i] - mx, dy = ys[i] - my, dz = zs[i] - mz;
        sxx = fma(dx, dx, sxx); sxy = fma(dx, dy, sxy); sxz = fma(dx, dz, sxz);
        syy = fma(dy, dy, syy); syz = fma(dy, dz, syz); szz = fma(dz, dz, szz);
    }
    sxx = wave_sum(sxx); sxy = wave_sum(sxy); sxz = wave_sum(sxz);
    syy = wave_sum(syy); syz = wave_sum(syz); szz = wave_sum(szz);
    if (lane == 0) {
        uint64_t key = skeys[a];
        cN[c] = n;
        cmu[3 * c + 0] = mx; cmu[3 * c + 1] = my; cmu[3 * c + 2] = mz;
        cS[6 * c + 0] = sxx; cS[6 * c + 1] = sxy; cS[6 * c + 2] = sxz;
        cS[6 * c + 3] = syy; cS[6 * c + 4] = syz; cS[6 * c + 5] = szz;
        cvox[c] = (int32_t)(key / (uint64_t)n_scans);
        cscan[c] = (int32_t)(key % (uint64_t)n_scans);
    }
}

__global__ void k_validate_sums(int64_t n, const int32_t *__restrict__ voxel, const int32_t *__restrict__ scan,
                                const int64_t *__restrict__ count, const double *__restrict__ s1,
                                const double *__restrict__ s2, int32_t n_scans, int32_t n_voxels,
                                int32_t *__restrict__ err) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int bad = 0;
    if (scan[i] < 0 || scan[i] >= n_scans) bad |= 2;
    if (voxel[i] < 0 || voxel[i] >= n_voxels) bad |= 4;
    if (count[i] < 1) bad |= 8;
    for (int k = 0; k < 3; k++) if (!isfinite(s1[3 * i + k])) bad |= 1;
    for (int k = 0; k < 6; k++) if (!isfinite(s2[6 * i + k])) bad |= 1;
    if (bad) atomicOr(err, bad);
}

__global__ void k_dup_keys(int64_t n, const uint64_t *__restrict__ keys, int32_t *__restrict__ err) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || i == 0) return;
    if (keys[i] == keys[i - 1]) atomicOr(err, 16);
}

// Centre raw sums once in double-double: mu = s / N, S = Q - s s^T / N.
__device__ __forceinline__ double centre_entry(double q, double sa, double sb, double n) {
    double ph = sa * sb;
    double pl = fma(sa, sb, -ph);
    double qh = ph / n;
    double rem = fma(-qh, n, ph) + pl;
    double ql = rem / n;
    double s, e;
    two_sum(q, -qh, s, e);
    return s + (e - ql);
}

__global__ void k_center_sums(int64_t C, const uint32_t *__restrict__ order, const uint64_t *__restrict__ skeys,
                              const int64_t *__restrict__ count, const double *__restrict__ s1,
                              const double *__restrict__ s2, int32_t n_scans, double *__restrict__ cN,
                              double *__restrict__ cmu, double *__restrict__ cS, int32_t *__restrict__ cvox,
                              int32_t *__restrict__ cscan) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    uint32_t j = order[c];
    double n = (double)count[j];
    double s[3] = {s1[3 * (int64_t)j], s1[3 * (int64_t)j + 1], s1[3 * (int64_t)j + 2]};
    for (int k = 0; k < 3; k++) {
        double q = s[k] / n;
        double r = fma(-q, n, s[k]);
        cmu[3 * c + k] = q + r / n;
    }
    const double *Q = s2 + 6 * (int64_t)j;
    cS[6 * c + 0] = centre_entry(Q[0], s[0], s[0], n);
    cS[6 * c + 1] = centre_entry(Q[1], s[0], s[1], n);
    cS[6 * c + 2] = centre_entry(Q[2], s[0], s[2], n);
    cS[6 * c + 3] = centre_entry(Q[3], s[1], s[1], n);
    cS[6 * c + 4] = centre_entry(Q[4], s[1], s[2], n);
    cS[6 * c + 5] = centre_entry(Q[5], s[2], s[2], n);
    cN[c] = n;
    uint64_t key = skeys[c];
    cvox[c] = (int32_t)(key / (uint64_t)n_scans);
    cscan[c] = (int32_t)(key % (uint64_t)n_scans);
}

// Scatter centred clusters into the voxel-major wave-interleaved layout.
__global__ void k_scatter_vox(int64_t C, const int64_t *__restrict__ dst, int64_t c_pad,
                              const double *__restrict__ cN, const double *__restrict__ cmu,
                              const double *__restrict__ cS, const int32_t *__restrict__ cscan,
                              double *__restrict__ vN, double *__restrict__ vmu, double *__restrict__ vS,
                              int32_t *__restrict__ vpose) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    int64_t d = dst[c];
    vN[d] = cN[c];
    vpose[d] = cscan[c];
#pragma unroll
    for (int k = 0; k < 3; k++) vmu[k * c_pad + d] = cmu[3 * c + k];
#pragma unroll
    for (int k = 0; k < 6; k++) vS[k * c_pad + d] = cS[6 * c + k];
}

// Gather centred clusters into the pose-major layout.
__global__ void k_gather_pose(int64_t C, const int32_t *__restrict__ order, const int32_t *__restrict__ slot_of,
                              const double *__restrict__ cN, const double *__restrict__ cmu,
                              const double *__restrict__ cS, double *__restrict__ pN, double *__restrict__ pmu,
                              double *__restrict__ pS, int32_t *__restrict__ pslot) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= C) return;
    int64_t c = order[q];
    pN[q] = cN[c];
    pslot[q] = slot_of[c];
#pragma unroll
    for (int k = 0; k < 3; k++) pmu[k * C + q] = cmu[3 * c + k];
#pragma unroll
    for (int k = 0; k < 6; k++) pS[k * C + q] = cS[6 * c + k];
}

static inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// ---------------------------------------------------------------- precision form
// Reference point of each voxel slot: the FP64 centroid c_i of the voxel's
// clusters placed by the reference poses T0.  Each cluster is then stored in
// FP32 in the world frame of its scan's reference pose, relative to c_i:
//   mu' = R0 mu + t0 - c_i,   S' = R0 S R0^T,
// so that at poses T the iteration only applies the pose change
// G = R R0^T = I + E (small) to small, voxel-centred quantities.
__device__ __forceinline__ void ref_frame_f32(const Pose &P0, const double *c, const double *mu, const double *S,
                                              float *mu32, float *S32) {
    double y[3], St[6];
    rot(P0.r, mu, y);
#pragma unroll
    for (int k = 0; k < 3; k++) mu32[k] = (float)((y[k] + P0.t[k]) - c[k]);
    rot_sym(P0.r, S, St);
#pragma unroll
    for (int k = 0; k < 6; k++) S32[k] = (float)St[k];
}

// One thread per slot; padding slots get a zero reference (their clusters are
// never read).  err: 1 = non-finite reference, 2 = a count >= 2^24.
__global__ void k_vox_ref_f32(int64_t n_slots, const GroupDesc *__restrict__ groups, int64_t c_pad,
                              const double *__restrict__ vN, const double *__restrict__ vmu,
                              const double *__restrict__ vS, const int32_t *__restrict__ vpose,
                              const double *__restrict__ ref_poses, double *__restrict__ vref,
                              float *__restrict__ vN32, float *__restrict__ vmu32, float *__restrict__ vS32,
                              int32_t *__restrict__ err) {
    const int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (sl >= n_slots) return;
    const GroupDesc g = groups[sl >> 6];
    const int lane = (int)(sl & 63);
    double *ref = vref + 4 * sl;
    if (lane >= g.nvox) {
        ref[0] = ref[1] = ref[2] = ref[3] = 0.0;
        return;
    }
    double n = 0.0, c[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < g.m; k++) {
        const int64_t idx = g.cbase + 64LL * k + lane;
        Pose P0;
        load_pose(ref_poses, vpose[idx], P0);
        const double mu[3] = {vmu[idx], vmu[c_pad + idx], vmu[2 * c_pad + idx]};
        double y[3];
        rot(P0.r, mu, y);
        const double nk = vN[idx];
        n += nk;
#pragma unroll
        for (int q = 0; q < 3; q++) c[q] = fma(nk, y[q] + P0.t[q], c[q]);
    }
#pragma unroll
    for (int q = 0; q < 3; q++) c[q] /= n;
    int bad = 0;
    if (!(isfinite(c[0]) && isfinite(c[1]) && isfinite(c[2]))) bad |= 1;
    ref[0] = c[0]; ref[1] = c[1]; ref[2] = c[2]; ref[3] = 0.0;
    for (int k = 0; k < g.m; k++) {
        const int64_t idx = g.cbase + 64LL * k + lane;
        Pose P0;
        load_pose(ref_poses, vpose[idx], P0);
        const double mu[3] = {vmu[idx], vmu[c_pad + idx], vmu[2 * c_pad + idx]};
        double S[6];
#pragma unroll
        for (int e = 0; e < 6; e++) S[e] = vS[e * c_pad + idx];
        float m32[3], S32[6];
        ref_frame_f32(P0, c, mu, S, m32, S32);
#pragma unroll
        for (int e = 0; e < 3; e++) vmu32[e * c_pad + idx] = m32[e];
#pragma unroll
        for (int e = 0; e < 6; e++) vS32[e * c_pad + idx] = S32[e];
        const double nk = vN[idx];
        if (nk >= 16777216.0) bad |= 2;
        vN32[idx] = (float)nk;
    }
    if (bad) atomicOr(err, bad);
}

// Pose-major FP32 copy in the same reference frames.
__global__ void k_gather_pose_f32(int64_t C, const int32_t *__restrict__ order, const int32_t *__restrict__ slot_of,
                                  const int32_t *__restrict__ cscan, const double *__restrict__ cN,
                                  const double *__restrict__ cmu, const double *__restrict__ cS,
                                  const double *__restrict__ vref, const double *__restrict__ ref_poses,
                                  float *__restrict__ pN, float *__restrict__ pmu, float *__restrict__ pS,
                                  int32_t *__restrict__ pslot) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= C) return;
    const int64_t c = order[q];
    const int32_t sl = slot_of[c];
    Pose P0;
    load_pose(ref_poses, cscan[c], P0);
    const double mu[3] = {cmu[3 * c], cmu[3 * c + 1], cmu[3 * c + 2]};
    double S[6];
#pragma unroll
    for (int k = 0; k < 6; k++) S[k] = cS[6 * c + k];
    float m32[3], S32[6];
    ref_frame_f32(P0, vref + 4LL * sl, mu, S, m32, S32);
#pragma unroll
    for (int k = 0; k < 3; k++) pmu[k * C + q] = m32[k];
#pragma unroll
    for (int k = 0; k < 6; k++) pS[k * C + q] = S32[k];
    pN[q] = (float)cN[c];
    pslot[q] = sl;
}

__global__ void k_validate_poses(int64_t n, const double *__restrict__ poses, int32_t *__restrict__ err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !isfinite(poses[i])) atomicOr(err, 1);
}


static int bit_length(uint64_t v) {
    int b = 0;
    while (v) { b++; v >>= 1; }
    return b;
}

// ---------------------------------------------------------------- pose chunks
// Cuts every pose's range of the pose-major layout into chunks of at most
// chunk_len clusters and uploads the chunk tables (synchronous).
ba_status replan_chunks(Problem *P, int32_t chunk_len, hipStream_t s) {
    if (chunk_len < MIN_CHUNK || chunk_len > MAX_CHUNK) {
        set_error("chunk_len %d out of range [%d, %d]", chunk_len, MIN_CHUNK, MAX_CHUNK);
        return BA_E_ARG;
    }
    const int32_t N = P->n_poses;
    std::vector<ChunkDesc> chunks;
    std::vector<int32_t> chunk_ptr(N + 1, 0);
    for (int32_t j = 0; j < N; j++) {
        chunk_ptr[j] = (int32_t)chunks.size();
        const int64_t a = P->h_pose_start[j], b = P->h_pose_start[j + 1];
        for (int64_t s0 = a; s0 < b; s0 += chunk_len) {
            ChunkDesc ch;
            ch.start = s0;
            ch.count = (int32_t)std::min<int64_t>(chunk_len, b - s0);
            ch.pose = j;
            chunks.push_back(ch);
        }
    }
    chunk_ptr[N] = (int32_t)chunks.size();
    if ((int64_t)chunks.size() > P->chunk_cap) {
        set_error("internal: %zu chunks exceed the table capacity %lld", chunks.size(), (long long)P->chunk_cap);
        return BA_E_ARG;
    }
    if (!chunks.empty())
        BA_HIP(hipMemcpyAsync(P->chunks, chunks.data(), sizeof(ChunkDesc) * chunks.size(), hipMemcpyHostToDevice, s));
    BA_HIP(hipMemcpyAsync(P->chunk_ptr, chunk_ptr.data(), sizeof(int32_t) * (N + 1), hipMemcpyHostToDevice, s));
    BA_HIP(hipStreamSynchronize(s));
    P->n_chunks = (int32_t)chunks.size();
    P->chunk_len = chunk_len;
    P->tune.chunk_len = chunk_len;
    return BA_OK;
}

// ---------------------------------------------------------------- host plan
// Builds every static table from the cluster labels (voxel-major order).
static ba_status make_plan(Problem *P, const std::vector<int32_t> &cvox, const std::vector<int32_t> &cscan,
                           const std::vector<int32_t> &scan_window, DevArena &keep, hipStream_t s) {
    const int64_t C = (int64_t)cvox.size();
    const int32_t N = P->n_poses;
    const int32_t W = P->n_windows;
    // voxel runs
    std::vector<int64_t> vstart;
    vstart.reserve((size_t)C / 2 + 2);
    for (int64_t c = 0; c < C; c++)
        if (c == 0 || cvox[c] != cvox[c - 1]) vstart.push_back(c);
    const int32_t V = (int32_t)vstart.size();
    vstart.push_back(C);
    P->n_vox = V;
    std::vector<int32_t> m(V), minpose(V), win(V);
    int32_t max_m = 0;
    for (int32_t v = 0; v < V; v++) {
        m[v] = (int32_t)(vstart[v + 1] - vstart[v]);
        minpose[v] = cscan[vstart[v]];
        win[v] = scan_window[minpose[v]];
        for (int64_t c = vstart[v]; c < vstart[v + 1]; c++)
            if (scan_window[cscan[c]] != win[v]) {
                set_error("voxel %d is observed by scans of different windows", cvox[vstart[v]]);
                return BA_E_ARG;
            }
        max_m = std::max(max_m, m[v]);
    }
    P->max_m = max_m;
    // voxel order: (window, m, first observing scan, voxel id), by three
    // stable counting passes (first scan, then m, then window)
    std::vector<int32_t> vorder(V);
    {
        std::vector<int32_t> other(V);
        std::iota(other.begin(), other.end(), 0);
        auto pass = [&](const std::vector<int32_t> &key, int32_t nkeys, const std::vector<int32_t> &in,
                        std::vector<int32_t> &out) {
            std::vector<int32_t> cnt((size_t)nkeys + 1, 0);
            for (int32_t i = 0; i < V; i++) cnt[key[in[i]] + 1]++;
            for (int32_t k = 0; k < nkeys; k++) cnt[k + 1] += cnt[k];
            for (int32_t i = 0; i < V; i++) out[cnt[key[in[i]]]++] = in[i];
        };
        pass(minpose, N, other, vorder);
        pass(m, max_m + 1, vorder, other);
        pass(win, W, other, vorder);
    }
    // wave groups: runs of up to 64 voxels of one window and one m in that
    // order; the group and lane of every voxel, then the clusters' places in
    // one pass over the clusters
    std::vector<GroupDesc> groups;
    std::vector<int32_t> win_group_ptr(W + 1, 0);
    std::vector<int64_t> dst(C);
    std::vector<int32_t> slot_of(C);
    std::vector<int32_t> slot_vox;
    std::vector<int32_t> gv(V), lv(V);
    int64_t cbase = 0;
    for (int32_t i = 0; i < V;) {
        int32_t j = i;
        while (j < V && win[vorder[j]] == win[vorder[i]] && m[vorder[j]] == m[vorder[i]] && j - i < 64) j++;
        GroupDesc g;
        g.cbase = cbase;
        g.m = m[vorder[i]];
        g.nvox = j - i;
        g.window = win[vorder[i]];
        g.scan0 = N;
        g.nscan = 0;
        g.pad = 0;
        const int32_t gi = (int32_t)groups.size();
        for (int32_t l = 0; l < 64; l++) slot_vox.push_back(l < g.nvox ? cvox[vstart[vorder[i + l]]] : -1);
        for (int32_t l = 0; l < g.nvox; l++) {
            gv[vorder[i + l]] = gi;
            lv[vorder[i + l]] = l;
        }
        groups.push_back(g);
        win_group_ptr[g.window + 1] = (int32_t)groups.size();
        cbase += 64LL * g.m;
        i = j;
    }
    {
        std::vector<int32_t> s1(groups.size(), -1);
        for (int32_t v = 0; v < V; v++) {
            GroupDesc &g = groups[gv[v]];
            const int32_t l = lv[v];
            for (int64_t c = vstart[v], k = 0; c < vstart[v + 1]; c++, k++) {
                dst[c] = g.cbase + 64LL * k + l;
                slot_of[c] = gv[v] * 64 + l;
                g.scan0 = std::min(g.scan0, cscan[c]);
                s1[gv[v]] = std::max(s1[gv[v]], cscan[c]);
            }
        }
        for (size_t gi = 0; gi < groups.size(); gi++) groups[gi].nscan = s1[gi] - groups[gi].scan0 + 1;
    }
    for (int32_t w = 0; w < W; w++) win_group_ptr[w + 1] = std::max(win_group_ptr[w + 1], win_group_ptr[w]);
    P->n_groups = (int32_t)groups.size();
    P->c_pad = cbase;
    // residual-pass blocks, one per group, the largest cluster counts first so
    // that the longest blocks start earliest
    std::vector<VoxBlock> vblocks;
    for (int32_t w = 0; w < W; w++)
        for (int32_t gi = win_group_ptr[w + 1] - 1; gi >= win_group_ptr[w]; gi--)
            vblocks.push_back(VoxBlock{gi, 1, 4, w});
    P->n_vblocks = (int32_t)vblocks.size();
    // the same groups with a split chosen per group: one wave up to 4
    // clusters per voxel, two up to 8, four beyond, so that no wave walks more
    // than about five clusters; a 256-thread block takes four one-wave, two
    // two-wave or one four-wave group of one window, largest counts first
    std::vector<VoxBlock> vmix;
    for (int32_t w = 0; w < W; w++) {
        int32_t gi = win_group_ptr[w + 1] - 1;
        while (gi >= win_group_ptr[w]) {
            const int32_t m = groups[gi].m;
            const int32_t sp = m <= 4 ? 1 : (m <= 8 ? 2 : 4);
            int32_t ng = 0;
            // groups gi, gi-1, ... of the same split (counts are non-increasing downwards)
            while (ng < 4 / sp && gi - ng >= win_group_ptr[w]) {
                const int32_t mm = groups[gi - ng].m;
                if ((mm <= 4 ? 1 : (mm <= 8 ? 2 : 4)) != sp) break;
                ng++;
            }
            vmix.push_back(VoxBlock{gi - ng + 1, ng, sp, w});
            gi -= ng;
        }
    }
    P->n_vblocks_mix = (int32_t)vmix.size();
    // pose-major order (scan, slot): a stable counting sort by scan of the
    // clusters listed in slot order (a voxel's clusters have distinct scans)
    std::vector<int32_t> porder(C);
    {
        std::vector<int32_t> by_slot(C);
        {
            std::vector<int64_t> slot_first(P->n_groups * 64LL + 1, 0);
            for (int64_t c = 0; c < C; c++) slot_first[slot_of[c] + 1]++;
            for (size_t i = 1; i < slot_first.size(); i++) slot_first[i] += slot_first[i - 1];
            for (int64_t c = 0; c < C; c++) by_slot[slot_first[slot_of[c]]++] = (int32_t)c;
        }
        std::vector<int64_t> scan_first(N + 1, 0);
        for (int64_t c = 0; c < C; c++) scan_first[cscan[c] + 1]++;
        for (int32_t j = 0; j < N; j++) scan_first[j + 1] += scan_first[j];
        for (int64_t q = 0; q < C; q++) {
            const int32_t c = by_slot[q];
            porder[scan_first[cscan[c]]++] = c;
        }
    }
    P->h_pose_start.assign(N + 1, 0);
    {
        int64_t q = 0;
        for (int32_t j = 0; j < N; j++) {
            P->h_pose_start[j] = q;
            while (q < C && cscan[porder[q]] == j) q++;
        }
        P->h_pose_start[N] = q;
    }
    P->chunk_cap = C / MIN_CHUNK + N + 1;
    std::vector<int32_t> win_pose_ptr(W + 1, 0), pose_window(N);
    for (int32_t j = 0; j < N; j++) {
        pose_window[j] = scan_window[j];
        win_pose_ptr[scan_window[j] + 1] = j + 1;
    }
    for (int32_t w = 0; w < W; w++) win_pose_ptr[w + 1] = std::max(win_pose_ptr[w + 1], win_pose_ptr[w]);

    // device allocations owned by the problem
    const int64_t CP = P->c_pad;
    const int64_t NS = (int64_t)P->n_groups * 64;
    // a precision-form problem keeps only FP32 iteration copies: the FP64
    // voxel-major copy is a build temporary and no FP64 pose-major copy exists
    const bool f32 = P->prec == BA_PREC_F32;
    DevArena f64tmp;
    DevArena &iter = f32 ? f64tmp : keep;
    BA_TRY(iter.alloc(&P->v_mu, 3 * CP));
    BA_TRY(iter.alloc(&P->v_S, 6 * CP));
    BA_TRY(iter.alloc(&P->v_N, CP));
    BA_TRY(keep.alloc(&P->v_pose, CP));
    BA_TRY(keep.alloc(&P->groups, std::max<int64_t>(P->n_groups, 1)));
    BA_TRY(keep.alloc(&P->vblocks, std::max<int64_t>(P->n_vblocks, 1)));
    BA_TRY(keep.alloc(&P->vblocks_mix, std::max<int64_t>(P->n_vblocks_mix, 1)));
    BA_TRY(keep.alloc(&P->slot_vox, std::max<int64_t>(NS, 1)));
    BA_TRY(keep.alloc(&P->vstate, 2 * std::max<int64_t>(NS, 1) * VSTATE));
    BA_TRY(keep.alloc(&P->wave_cost, std::max<int64_t>(P->n_groups, 1)));
    if (f32) {
        BA_TRY(keep.alloc(&P->v_mu32, 3 * CP));
        BA_TRY(keep.alloc(&P->v_S32, 6 * CP));
        BA_TRY(keep.alloc(&P->v_N32, CP));
        BA_TRY(keep.alloc(&P->p_mu32, 3 * C));
        BA_TRY(keep.alloc(&P->p_S32, 6 * C));
        BA_TRY(keep.alloc(&P->p_N32, C));
        BA_TRY(keep.alloc(&P->v_ref, 4 * std::max<int64_t>(NS, 1)));
        BA_TRY(keep.alloc(&P->pdelta, 16LL * N));
    } else {
        BA_TRY(keep.alloc(&P->p_mu, 3 * C));
        BA_TRY(keep.alloc(&P->p_S, 6 * C));
        BA_TRY(keep.alloc(&P->p_N, C));
    }
    BA_TRY(keep.alloc(&P->p_slot, C));
    BA_TRY(keep.alloc(&P->p_cidx, C));
    BA_TRY(keep.alloc(&P->chunks, P->chunk_cap));
    BA_TRY(keep.alloc(&P->chunk_ptr, N + 1));
    BA_TRY(keep.alloc(&P->partials, P->chunk_cap * NPART));
    BA_TRY(keep.alloc(&P->win_group_ptr, W + 1));
    BA_TRY(keep.alloc(&P->win_pose_ptr, W + 1));
    BA_TRY(keep.alloc(&P->pose_window, N));
    BA_TRY(keep.alloc(&P->g, 6LL * N));
    BA_TRY(keep.alloc(&P->H, 36LL * N));
    BA_TRY(keep.alloc(&P->dx, 6LL * N));
    BA_TRY(keep.alloc(&P->poses_trial, 12LL * N));
    BA_TRY(keep.alloc(&P->pose_q, N));
    BA_TRY(keep.alloc(&P->pose_info, N));
    BA_TRY(keep.alloc(&P->lm, W));
    P->h_win_pose_ptr = new int32_t[W + 1];
    std::memcpy(P->h_win_pose_ptr, win_pose_ptr.data(), sizeof(int32_t) * (W + 1));

    BA_HIP(hipMemsetAsync(P->v_mu, 0, sizeof(double) * 3 * CP, s));
    BA_HIP(hipMemsetAsync(P->v_S, 0, sizeof(double) * 6 * CP, s));
    BA_HIP(hipMemsetAsync(P->v_N, 0, sizeof(double) * CP, s));
    BA_HIP(hipMemsetAsync(P->v_pose, 0, sizeof(int32_t) * CP, s));
    BA_HIP(hipMemsetAsync(P->vstate, 0, sizeof(double) * 2 * std::max<int64_t>(NS, 1) * VSTATE, s));
    BA_HIP(hipMemcpyAsync(P->groups, groups.data(), sizeof(GroupDesc) * groups.size(), hipMemcpyHostToDevice, s));
    BA_HIP(hipMemcpyAsync(P->vblocks, vblocks.data(), sizeof(VoxBlock) * vblocks.size(), hipMemcpyHostToDevice, s));
    if (!vmix.empty())
        BA_HIP(hipMemcpyAsync(P->vblocks_mix, vmix.data(), sizeof(VoxBlock) * vmix.size(), hipMemcpyHostToDevice, s));
    BA_HIP(hipMemcpyAsync(P->slot_vox, slot_vox.data(), sizeof(int32_t) * slot_vox.size(), hipMemcpyHostToDevice, s));
    BA_TRY(replan_chunks(P, P->chunk_len, s));
    BA_HIP(hipMemcpyAsync(P->win_group_ptr, win_group_ptr.data(), sizeof(int32_t) * (W + 1), hipMemcpyHostToDevice, s));
    BA_HIP(hipMemcpyAsync(P->win_pose_ptr, win_pose_ptr.data(), sizeof(int32_t) * (W + 1), hipMemcpyHostToDevice, s));
    BA_HIP(hipMemcpyAsync(P->pose_window, pose_window.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice, s));

    // scatter / gather the cluster payload
    DevArena tmp;
    int64_t *d_dst;
    int32_t *d_slot_of, *d_porder;
    BA_TRY(tmp.alloc(&d_dst, C));
    BA_TRY(keep.alloc(&P->c_slot, C));
    d_slot_of = P->c_slot;
    BA_TRY(tmp.alloc(&d_porder, C));
    int32_t *d_err;
    BA_TRY(tmp.alloc(&d_err, 1));
    BA_HIP(hipMemcpyAsync(d_dst, dst.data(), sizeof(int64_t) * C, hipMemcpyHostToDevice, s));
    BA_HIP(hipMemcpyAsync(d_slot_of, slot_of.data(), sizeof(int32_t) * C, hipMemcpyHostToDevice, s));
    BA_HIP(hipMemcpyAsync(d_porder, porder.data(), sizeof(int32_t) * C, hipMemcpyHostToDevice, s));
    BA_HIP(hipMemcpyAsync(P->p_cidx, porder.data(), sizeof(int32_t) * C, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_scatter_vox, dim3(nblk(C)), dim3(256), 0, s, C, d_dst, CP, P->c_N, P->c_mu, P->c_S,
                       P->c_scan, P->v_N, P->v_mu, P->v_S, P->v_pose);
    if (!f32) {
        hipLaunchKernelGGL(k_gather_pose, dim3(nblk(C)), dim3(256), 0, s, C, d_porder, d_slot_of, P->c_N, P->c_mu,
                           P->c_S, P->p_N, P->p_mu, P->p_S, P->p_slot);
        BA_HIP(hipGetLastError());
        BA_HIP(hipStreamSynchronize(s));
        return BA_OK;
    }
    BA_HIP(hipMemsetAsync(d_err, 0, sizeof(int32_t), s));
    BA_HIP(hipMemsetAsync(P->v_mu32, 0, sizeof(float) * 3 * CP, s));
    BA_HIP(hipMemsetAsync(P->v_S32, 0, sizeof(float) * 6 * CP, s));
    BA_HIP(hipMemsetAsync(P->v_N32, 0, sizeof(float) * CP, s));
    if (NS > 0)
        hipLaunchKernelGGL(k_vox_ref_f32, dim3(nblk(NS)), dim3(256), 0, s, NS, P->groups, CP, P->v_N, P->v_mu, P->v_S,
                           P->v_pose, P->ref_poses, P->v_ref, P->v_N32, P->v_mu32, P->v_S32, d_err);
    hipLaunchKernelGGL(k_gather_pose_f32, dim3(nblk(C)), dim3(256), 0, s, C, d_porder, d_slot_of, P->c_scan,
                       P->c_N, P->c_mu, P->c_S, P->v_ref, P->ref_poses, P->p_N32, P->p_mu32, P->p_S32, P->p_slot);
    BA_HIP(hipGetLastError());
    int32_t herr = 0;
    BA_HIP(hipMemcpyAsync(&herr, d_err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BA_HIP(hipStreamSynchronize(s));
    P->v_mu = P->v_S = P->v_N = nullptr;   // released with f64tmp
    if (herr & 2) {
        set_error("precision form: a cluster holds 2^24 points or more (its count is not exact in FP32)");
        return BA_E_UNSUPPORTED;
    }
    if (herr & 1) {
        set_error("precision form: non-finite voxel reference point (check ref_poses)");
        return BA_E_ARG;
    }
    return BA_OK;
}

static ba_status finish_build(Problem *P, DevArena &keep, const ba_build_options *opt, hipStream_t s) {
    const int64_t C = P->n_clusters;
    std::vector<int32_t> cvox(C), cscan(C);
    BA_HIP(hipMemcpyAsync(cvox.data(), P->c_vox, sizeof(int32_t) * C, hipMemcpyDeviceToHost, s));
    BA_HIP(hipMemcpyAsync(cscan.data(), P->c_scan, sizeof(int32_t) * C, hipMemcpyDeviceToHost, s));
    BA_HIP(hipStreamSynchronize(s));
    std::vector<int32_t> scan_window(P->n_poses, 0);
    int32_t W = 1;
    if (opt && opt->n_windows > 1) {
        if (!opt->scan_window) {
            set_error("n_windows > 1 needs scan_window");
            return BA_E_ARG;
        }
        W = opt->n_windows;
        for (int32_t j = 0; j < P->n_poses; j++) {
            int32_t w = opt->scan_window[j];
            if (w < 0 || w >= W || (j > 0 && w < scan_window[j - 1])) {
                set_error("scan_window must be non-decreasing in [0, n_windows)");
                return BA_E_ARG;
            }
            scan_window[j] = w;
        }
    }
    P->n_windows = W;
    P->prec = opt ? opt->precision : BA_PREC_F64;
    if (P->prec != BA_PREC_F64 && P->prec != BA_PREC_F32) {
        set_error("unknown precision %d", P->prec);
        return BA_E_ARG;
    }
    if (P->prec == BA_PREC_F32) {
        if (!opt->ref_poses) {
            set_error("the precision form needs ref_poses");
            return BA_E_ARG;
        }
        const int64_t np = 12LL * P->n_poses;
        BA_TRY(keep.alloc(&P->ref_poses, np));
        BA_HIP(hipMemcpyAsync(P->ref_poses, opt->ref_poses, sizeof(double) * np, hipMemcpyDeviceToDevice, s));
        DevArena tmp;
        int32_t *d_err;
        BA_TRY(tmp.alloc(&d_err, 1));
        BA_HIP(hipMemsetAsync(d_err, 0, sizeof(int32_t), s));
        hipLaunchKernelGGL(k_validate_poses, dim3(nblk(np)), dim3(256), 0, s, np, P->ref_poses, d_err);
        BA_HIP(hipGetLastError());
        int32_t herr = 0;
        BA_HIP(hipMemcpyAsync(&herr, d_err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        BA_HIP(hipStreamSynchronize(s));
        if (herr) {
            set_error("ref_poses holds non-finite values");
            return BA_E_ARG;
        }
    }
    return make_plan(P, cvox, cscan, scan_window, keep, s);
}

ba_status build_from_points(const ba_points *pts, const ba_build_options *opt, Problem *P, DevArena &keep,
                            hipStream_t s) {
    const int64_t n = pts->n;
    if (n < 1 || n > (int64_t)0xFFFFFFFF) {
        set_error("point count %lld out of range [1, 2^32)", (long long)n);
        return BA_E_ARG;
    }
    if (!pts->x || !pts->y || !pts->z || !pts->scan || !pts->voxel || pts->n_scans < 1 || pts->n_voxels < 1) {
        set_error("null point array or empty label range");
        return BA_E_ARG;
    }
    P->n_poses = pts->n_scans;
    P->n_voxels_in = pts->n_voxels;
    P->chunk_len = (opt && opt->chunk_len > 0) ? opt->chunk_len : 256;
    DevArena tmp;
    int32_t *err;
    uint64_t *keys;
    uint32_t *vals;
    int64_t *flags, *total;
    BA_TRY(tmp.alloc(&err, 1));
    BA_TRY(tmp.alloc(&keys, n));
    BA_TRY(tmp.alloc(&vals, n));
    BA_TRY(tmp.alloc(&flags, n + 1));
    BA_TRY(tmp.alloc(&total, 1));
    size_t ws_bytes = std::max(radix_sort_workspace_bytes(n), scan_workspace_bytes(n));
    char *ws;
    BA_TRY(tmp.alloc(&ws, (int64_t)ws_bytes));
    BA_HIP(hipMemsetAsync(err, 0, sizeof(int32_t), s));
    hipLaunchKernelGGL(k_validate_points, dim3(nblk(n)), dim3(256), 0, s, n, pts->x, pts->y, pts->z, pts->scan,
                       pts->voxel, pts->n_scans, pts->n_voxels, err);
    hipLaunchKernelGGL(k_make_keys, dim3(nblk(n)), dim3(256), 0, s, n, pts->scan, pts->voxel, pts->n_scans, keys,
                       vals);
    BA_HIP(hipGetLastError());
    int32_t herr = 0;
    BA_HIP(hipMemcpyAsync(&herr, err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BA_HIP(hipStreamSynchronize(s));
    if (herr) {
        set_error("invalid points (flags 0x%x: 1 non-finite, 2 scan out of range, 4 voxel out of range)", herr);
        return BA_E_ARG;
    }
    int bits = bit_length((uint64_t)pts->n_voxels * (uint64_t)pts->n_scans - 1);
    BA_HIP(radix_sort_pairs(keys, vals, n, bits, ws, s));
    hipLaunchKernelGGL(k_head_flags, dim3(nblk(n)), dim3(256), 0, s, n, keys, flags);
    BA_HIP(exclusive_scan_i64(flags, flags, n, total, ws, s));
    int64_t C = 0;
    BA_HIP(hipMemcpyAsync(&C, total, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    BA_HIP(hipStreamSynchronize(s));
    P->n_clusters = C;
    int64_t *starts;
    double *xs, *ys, *zs;
    BA_TRY(tmp.alloc(&starts, C + 1));
    BA_TRY(tmp.alloc(&xs, n));
    BA_TRY(tmp.alloc(&ys, n));
    BA_TRY(tmp.alloc(&zs, n));
    hipLaunchKernelGGL(k_segment_starts, dim3(nblk(n)), dim3(256), 0, s, n, keys, flags, starts, C);
    hipLaunchKernelGGL(k_gather_xyz, dim3(nblk(n)), dim3(256), 0, s, n, vals, pts->x, pts->y, pts->z, xs, ys, zs);
    BA_TRY(keep.alloc(&P->c_N, C));
    BA_TRY(keep.alloc(&P->c_mu, 3 * C));
    BA_TRY(keep.alloc(&P->c_S, 6 * C));
    BA_TRY(keep.alloc(&P->c_vox, C));
    BA_TRY(keep.alloc(&P->c_scan, C));
    hipLaunchKernelGGL(k_cluster_stats, dim3(nblk(C * 64)), dim3(256), 0, s, C, starts, xs, ys, zs, keys,
                       pts->n_scans, P->c_N, P->c_mu, P->c_S, P->c_vox, P->c_scan);
    BA_HIP(hipGetLastError());
    return finish_build(P, keep, opt, s);
}

ba_status build_from_sums(const ba_cluster_sums *cs, const ba_build_options *opt, Problem *P, DevArena &keep,
                          hipStream_t s) {
    const int64_t n = cs->n;
    if (n < 1 || n > (int64_t)0xFFFFFFFF) {
        set_error("cluster count %lld out of range [1, 2^32)", (long long)n);
        return BA_E_ARG;
    }
    if (!cs->voxel || !cs->scan || !cs->count || !cs->sum || !cs->sumsq || cs->n_scans < 1 || cs->n_voxels < 1) {
        set_error("null cluster array or empty label range");
        return BA_E_ARG;
    }
    P->n_poses = cs->n_scans;
    P->n_voxels_in = cs->n_voxels;
    P->chunk_len = (opt && opt->chunk_len > 0) ? opt->chunk_len : 256;
    DevArena tmp;
    int32_t *err;
    uint64_t *keys;
    uint32_t *vals;
    BA_TRY(tmp.alloc(&err, 1));
    BA_TRY(tmp.alloc(&keys, n));
    BA_TRY(tmp.alloc(&vals, n));
    char *ws;
    BA_TRY(tmp.alloc(&ws, (int64_t)radix_sort_workspace_bytes(n)));
    BA_HIP(hipMemsetAsync(err, 0, sizeof(int32_t), s));
    hipLaunchKernelGGL(k_validate_sums, dim3(nblk(n)), dim3(256), 0, s, n, cs->voxel, cs->scan, cs->count, cs->sum,
                       cs->sumsq, cs->n_scans, cs->n_voxels, err);
    hipLaunchKernelGGL(k_make_keys, dim3(nblk(n)), dim3(256), 0, s, n, cs->scan, cs->voxel, cs->n_scans, keys, vals);
    int bits = bit_length((uint64_t)cs->n_voxels * (uint64_t)cs->n_scans - 1);
    BA_HIP(radix_sort_pairs(keys, vals, n, bits, ws, s));
    hipLaunchKernelGGL(k_dup_keys, dim3(nblk(n)), dim3(256), 0, s, n, keys, err);
    BA_HIP(hipGetLastError());
    int32_t herr = 0;
    BA_HIP(hipMemcpyAsync(&herr, err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BA_HIP(hipStreamSynchronize(s));
    if (herr) {
        set_error("invalid clusters (flags 0x%x: 1 non-finite, 2 scan, 4 voxel, 8 count < 1, 16 duplicate pair)",
                  herr);
        return BA_E_ARG;
    }
    P->n_clusters = n;
    BA_TRY(keep.alloc(&P->c_N, n));
    BA_TRY(keep.alloc(&P->c_mu, 3 * n));
    BA_TRY(keep.alloc(&P->c_S, 6 * n));
    BA_TRY(keep.alloc(&P->c_vox, n));
    BA_TRY(keep.alloc(&P->c_scan, n));
    hipLaunchKernelGGL(k_center_sums, dim3(nblk(n)), dim3(256), 0, s, n, vals, keys, cs->count, cs->sum, cs->sumsq,
                       cs->n_scans, P->c_N, P->c_mu, P->c_S, P->c_vox, P->c_scan);
    BA_HIP(hipGetLastError());
    return finish_build(P, keep, opt, s);
}

}  // namespace ba
