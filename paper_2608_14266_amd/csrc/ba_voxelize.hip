// Bottom-up multi-level voxelization and planarity selection (Sec. IV-A):
// points -> world cells at the finest edge d (Eq. 4) -> per (cell, scan)
// clusters (Eq. 2) -> L levels, each halving the previous level's cell
// indices (Eq. 5) and merging its clusters -> per-cell planarity test
// lambda0 < tau lambda1 on the voxel covariance at the given poses -> the kept
// cells of all levels concatenated (Alg. 1, BottomUpVoxelization, Selection).
//
//   k_vx_cells        world point and level-1 cell per point, block bounding
//                     boxes and error flags (grid-stride, fixed grid)
//   k_vx_bbox         one block: bounding box and flags of the whole cloud
//   k_vx_keys_points  packed (cell offsets, scan) key per point
//   k_vx_keys_up      packed key of the parent cell per cluster
//   (stable LSD radix sort of the keys, head flags, exclusive scan)
//   k_vx_sum_points   8 lanes per level-1 cluster: raw sums of its points
//   k_vx_sum_clusters thread per level-k cluster: sums of its child clusters
//   k_vx_select       thread per cell: voxel covariance, eigenvalues, decision
//   k_vx_emit         thread per kept cell: its clusters into the output
//
// Sums run in a fixed order (sorted position), so results are deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "ba.h"
#include "ba_device.hpp"
#include "ba_internal.hpp"

namespace ba {

static constexpr int VX_THREADS = 256;
static constexpr int VX_BOX_BLOCKS = 2048;
static constexpr int64_t VX_CELL_LIMIT = (int64_t)1 << 30;   // |cell index| bound at level 1
static constexpr double VX_RANK2 = 1e-10;                      // l1 / l2 below this: rank below two

static inline unsigned vx_nblk(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + VX_THREADS - 1) / VX_THREADS); }

static int vx_bit_length(uint64_t v) {
    int b = 0;
    while (v) {
        b++;
        v >>= 1;
    }
    return b;
}

// Packed key of a cell and scan at one level: offsets from the level's
// minimum cell in bits[0] + bits[1] + bits[2] high bits (x, y, z), the scan in
// the low sbits; integer order of keys is the (x, y, z, scan) order.
struct CellLayout {
    int64_t lo[3];
    int64_t hi[3];
    int bits[3];
    int sbits;
    int total;
};

static CellLayout make_layout(const int64_t lo[3], const int64_t hi[3], int32_t n_scans) {
    CellLayout L;
    for (int r = 0; r < 3; r++) {
        L.lo[r] = lo[r];
        L.hi[r] = hi[r];
        L.bits[r] = vx_bit_length((uint64_t)(hi[r] - lo[r]));
    }
    L.sbits = vx_bit_length((uint64_t)(n_scans - 1));
    L.total = L.bits[0] + L.bits[1] + L.bits[2] + L.sbits;
    return L;
}

// a field of zero width holds only the value 0 (and is never shifted by 64)
__device__ __forceinline__ uint64_t vx_field(uint64_t v, int width, int shift) {
    return width ? (v << shift) : 0;
}

__device__ __forceinline__ uint64_t vx_pack(const CellLayout &L, int64_t cx, int64_t cy, int64_t cz, int32_t s) {
    return vx_field((uint64_t)(cx - L.lo[0]), L.bits[0], L.bits[1] + L.bits[2] + L.sbits) |
           vx_field((uint64_t)(cy - L.lo[1]), L.bits[1], L.bits[2] + L.sbits) |
           vx_field((uint64_t)(cz - L.lo[2]), L.bits[2], L.sbits) | vx_field((uint64_t)s, L.sbits, 0);
}

__device__ __forceinline__ void vx_unpack(const CellLayout &L, uint64_t k, int64_t c[3], int32_t &s) {
    s = L.sbits ? (int32_t)(k & ((1ULL << L.sbits) - 1)) : 0;
    k = L.sbits ? (k >> L.sbits) : k;
    c[2] = L.lo[2] + (int64_t)(L.bits[2] ? (k & ((1ULL << L.bits[2]) - 1)) : 0);
    k = L.bits[2] ? (k >> L.bits[2]) : k;
    c[1] = L.lo[1] + (int64_t)(L.bits[1] ? (k & ((1ULL << L.bits[1]) - 1)) : 0);
    k = L.bits[1] ? (k >> L.bits[1]) : k;
    c[0] = L.lo[0] + (int64_t)(L.bits[0] ? k : 0);
}

// error flags of the cloud
static constexpr int VX_ERR_FINITE = 1, VX_ERR_SCAN = 2, VX_ERR_RANGE = 4;

__global__ __launch_bounds__(VX_THREADS) void k_vx_cells(int64_t n, const double *__restrict__ x,
                                                         const double *__restrict__ y, const double *__restrict__ z,
                                                         const int32_t *__restrict__ scan, int32_t n_scans,
                                                         const double *__restrict__ poses, double d,
                                                         int32_t *__restrict__ cell, int32_t *__restrict__ bpart) {
    // the world point is formed with every product and sum rounded on its own
    // (no fused multiply-add), so the cell decisions are reproducible
#pragma clang fp contract(off)
    constexpr int NW = VX_THREADS / 64;
    __shared__ int red[NW];
    int lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, nhi[3] = {INT32_MAX, INT32_MAX, INT32_MAX};
    int err = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t s = scan[i];
        if (s < 0 || s >= n_scans) {
            err |= VX_ERR_SCAN;
            continue;
        }
        const double *P = poses + 12LL * s;
        const double p[3] = {x[i], y[i], z[i]};
        int32_t c[3] = {0, 0, 0};
        bool ok = true;
#pragma unroll
        for (int r = 0; r < 3; r++) {
            const double w = ((P[3 * r] * p[0] + P[3 * r + 1] * p[1]) + P[3 * r + 2] * p[2]) + P[9 + r];
            const double f = floor(w / d);
            if (!(fabs(f) < (double)VX_CELL_LIMIT)) {
                err |= isfinite(f) ? VX_ERR_RANGE : VX_ERR_FINITE;
                ok = false;
            } else {
                c[r] = (int32_t)f;
            }
        }
        if (!ok) continue;
#pragma unroll
        for (int r = 0; r < 3; r++) {
            cell[(int64_t)r * n + i] = c[r];
            lo[r] = min(lo[r], c[r]);
            nhi[r] = min(nhi[r], -c[r]);
        }
    }
    int *out = bpart + 7LL * blockIdx.x;
#pragma unroll
    for (int r = 0; r < 3; r++) {
        const int a = block_min_i<NW>(lo[r], red);
        const int b = block_min_i<NW>(nhi[r], red);
        if (threadIdx.x == 0) {
            out[r] = a;
            out[3 + r] = b;
        }
    }
    // OR of the flags, one bit at a time (a bit is set if some thread's is)
    int orr = 0;
#pragma unroll
    for (int bit = 0; bit < 3; bit++) orr |= (block_min_i<NW>((err >> bit) & 1 ? 0 : 1, red) == 0) ? (1 << bit) : 0;
    if (threadIdx.x == 0) out[6] = orr;
}

__global__ __launch_bounds__(VX_THREADS) void k_vx_bbox(int nb, const int32_t *__restrict__ bpart,
                                                        int32_t *__restrict__ box) {
    constexpr int NW = VX_THREADS / 64;
    __shared__ int red[NW];
    int v[6] = {INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX};
    int flags = 0;
    for (int b = threadIdx.x; b < nb; b += VX_THREADS) {
#pragma unroll
        for (int q = 0; q < 6; q++) v[q] = min(v[q], bpart[7 * b + q]);
        flags |= bpart[7 * b + 6];
    }
#pragma unroll
    for (int q = 0; q < 6; q++) {
        const int m = block_min_i<NW>(v[q], red);
        if (threadIdx.x == 0) box[q] = m;
    }
    int orr = 0;
#pragma unroll
    for (int bit = 0; bit < 3; bit++) orr |= (block_min_i<NW>((flags >> bit) & 1 ? 0 : 1, red) == 0) ? (1 << bit) : 0;
    if (threadIdx.x == 0) box[6] = orr;
}

__global__ void k_vx_keys_points(int64_t n, const int32_t *__restrict__ cell, const int32_t *__restrict__ scan,
                                 CellLayout L, uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    keys[i] = vx_pack(L, cell[i], cell[n + i], cell[2 * n + i], scan[i]);
    vals[i] = (uint32_t)i;
}

// key of the parent cell (Eq. 5: floor of half the index) of each cluster
__global__ void k_vx_keys_up(int64_t C, const uint64_t *__restrict__ ckey, CellLayout Lc, CellLayout Lp,
                             uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= C) return;
    int64_t c[3];
    int32_t s;
    vx_unpack(Lc, ckey[i], c, s);
    keys[i] = vx_pack(Lp, c[0] >> 1, c[1] >> 1, c[2] >> 1, s);
    vals[i] = (uint32_t)i;
}

// head flag where (key >> shift) changes
__global__ void k_vx_heads(int64_t n, const uint64_t *__restrict__ keys, int shift, int64_t *__restrict__ flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    flags[i] = (i == 0 || (keys[i] >> shift) != (keys[i - 1] >> shift)) ? 1 : 0;
}

__global__ void k_vx_starts(int64_t n, const uint64_t *__restrict__ keys, int shift, const int64_t *__restrict__ excl,
                            int64_t *__restrict__ starts, int64_t n_seg) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (i == 0 || (keys[i] >> shift) != (keys[i - 1] >> shift)) starts[excl[i]] = i;
    if (i == 0) starts[n_seg] = n;
}

// raw sums of one level-1 cluster: VX_SUM_LANES lanes per cluster, lane g
// summing the points g, g + VX_SUM_LANES, ... of the cluster's sorted
// (stable) run, then the group adding its lanes' sums in a fixed tree
static constexpr int VX_SUM_LANES = 8;
__global__ void k_vx_sum_points(int64_t C, const int64_t *__restrict__ starts, const uint64_t *__restrict__ keys,
                                const uint32_t *__restrict__ idx, const double *__restrict__ x,
                                const double *__restrict__ y, const double *__restrict__ z,
                                uint64_t *__restrict__ ckey, int64_t *__restrict__ count, double *__restrict__ s1,
                                double *__restrict__ s2) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t c = tid / VX_SUM_LANES;
    const int g = (int)(tid % VX_SUM_LANES);
    double m[3] = {0, 0, 0}, q[6] = {0, 0, 0, 0, 0, 0};
    int64_t a = 0, b = 0;
    if (c < C) {
        a = starts[c];
        b = starts[c + 1];
        for (int64_t k = a + g; k < b; k += VX_SUM_LANES) {
            const uint32_t i = idx[k];
            const double p[3] = {x[i], y[i], z[i]};
#pragma unroll
            for (int r = 0; r < 3; r++) m[r] += p[r];
            q[0] = fma(p[0], p[0], q[0]);
            q[1] = fma(p[0], p[1], q[1]);
            q[2] = fma(p[0], p[2], q[2]);
            q[3] = fma(p[1], p[1], q[3]);
            q[4] = fma(p[1], p[2], q[4]);
            q[5] = fma(p[2], p[2], q[5]);
        }
    }
    // every lane takes part in the shuffles (groups are aligned within a wave)
#pragma unroll
    for (int o = VX_SUM_LANES / 2; o > 0; o >>= 1) {
#pragma unroll
        for (int r = 0; r < 3; r++) m[r] += __shfl_xor(m[r], o, VX_SUM_LANES);
#pragma unroll
        for (int r = 0; r < 6; r++) q[r] += __shfl_xor(q[r], o, VX_SUM_LANES);
    }
    if (c >= C || g != 0) return;
    ckey[c] = keys[a];
    count[c] = b - a;
#pragma unroll
    for (int r = 0; r < 3; r++) s1[3 * c + r] = m[r];
#pragma unroll
    for (int r = 0; r < 6; r++) s2[6 * c + r] = q[r];
}

// raw sums of one level-k cluster from its children (sorted, stable order)
__global__ void k_vx_sum_clusters(int64_t C, const int64_t *__restrict__ starts, const uint64_t *__restrict__ keys,
                                  const uint32_t *__restrict__ idx, const int64_t *__restrict__ cnt_in,
                                  const double *__restrict__ s1_in, const double *__restrict__ s2_in,
                                  uint64_t *__restrict__ ckey, int64_t *__restrict__ count, double *__restrict__ s1,
                                  double *__restrict__ s2) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    const int64_t a = starts[c], b = starts[c + 1];
    int64_t nn = 0;
    double m[3] = {0, 0, 0}, q[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t k = a; k < b; k++) {
        const uint32_t i = idx[k];
        nn += cnt_in[i];
#pragma unroll
        for (int r = 0; r < 3; r++) m[r] += s1_in[3LL * i + r];
#pragma unroll
        for (int r = 0; r < 6; r++) q[r] += s2_in[6LL * i + r];
    }
    ckey[c] = keys[a];
    count[c] = nn;
#pragma unroll
    for (int r = 0; r < 3; r++) s1[3 * c + r] = m[r];
#pragma unroll
    for (int r = 0; r < 6; r++) s2[6 * c + r] = q[r];
}

// Planarity of one cell: its clusters centred (mu = sum p / N,
// S = sum p p^T - mu (sum p)^T), mapped by their scans' poses, combined into
// the voxel covariance about the voxel mean (Eq. 1 in centred form), and the
// 3x3 eigenvalues; kept when l0 < tau l1, the cell holds at least three
// points and its covariance has rank two or more (l1 > VX_RANK2 l2): fewer
// points or a line span no plane, and their l1 is only rounding; and when
// enough scans observe it.
__global__ void k_vx_select(int64_t V, const int64_t *__restrict__ vstart, const uint64_t *__restrict__ ckey,
                            const int64_t *__restrict__ count, const double *__restrict__ s1,
                            const double *__restrict__ s2, CellLayout L, const double *__restrict__ poses, double tau,
                            int32_t min_scans, int64_t *__restrict__ keep, int64_t *__restrict__ kept_clusters,
                            double *__restrict__ lam_out) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    const int64_t a = vstart[v], b = vstart[v + 1];
    double Nv = 0.0, mw[3] = {0, 0, 0};
    for (int64_t c = a; c < b; c++) {
        int64_t cc[3];
        int32_t s;
        vx_unpack(L, ckey[c], cc, s);
        const double *P = poses + 12LL * s;
        const double n = (double)count[c];
        // N mu_w = R (sum p) + N t
#pragma unroll
        for (int r = 0; r < 3; r++)
            mw[r] += P[3 * r] * s1[3 * c] + P[3 * r + 1] * s1[3 * c + 1] + P[3 * r + 2] * s1[3 * c + 2] + n * P[9 + r];
        Nv += n;
    }
#pragma unroll
    for (int r = 0; r < 3; r++) mw[r] /= Nv;
    double A[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t c = a; c < b; c++) {
        int64_t cc[3];
        int32_t s;
        vx_unpack(L, ckey[c], cc, s);
        const double *P = poses + 12LL * s;
        const double n = (double)count[c];
        const double mu[3] = {s1[3 * c] / n, s1[3 * c + 1] / n, s1[3 * c + 2] / n};
        const double *q = s2 + 6 * c;
        const double S[3][3] = {{q[0] - mu[0] * s1[3 * c], q[1] - mu[0] * s1[3 * c + 1], q[2] - mu[0] * s1[3 * c + 2]},
                                {q[1] - mu[1] * s1[3 * c], q[3] - mu[1] * s1[3 * c + 1], q[4] - mu[1] * s1[3 * c + 2]},
                                {q[2] - mu[2] * s1[3 * c], q[4] - mu[2] * s1[3 * c + 1], q[5] - mu[2] * s1[3 * c + 2]}};
        double RS[3][3], dw[3];
#pragma unroll
        for (int i = 0; i < 3; i++) {
            dw[i] = P[3 * i] * mu[0] + P[3 * i + 1] * mu[1] + P[3 * i + 2] * mu[2] + P[9 + i] - mw[i];
#pragma unroll
            for (int j = 0; j < 3; j++)
                RS[i][j] = P[3 * i] * S[0][j] + P[3 * i + 1] * S[1][j] + P[3 * i + 2] * S[2][j];
        }
        int k = 0;
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int j = i; j < 3; j++) {
                const double sw = RS[i][0] * P[3 * j] + RS[i][1] * P[3 * j + 1] + RS[i][2] * P[3 * j + 2];
                A[k++] += sw + n * dw[i] * dw[j];
            }
    }
#pragma unroll
    for (int k = 0; k < 6; k++) A[k] /= Nv;
    double lam[3], u[3];
    eig_sym3(A, lam, u);
    const bool ok = Nv >= 3.0 && lam[1] > VX_RANK2 * lam[2] && lam[0] < tau * lam[1] &&
                    (b - a) >= (int64_t)min_scans;
    keep[v] = ok ? 1 : 0;
    kept_clusters[v] = ok ? (b - a) : 0;
    if (lam_out) {
#pragma unroll
        for (int r = 0; r < 3; r++) lam_out[3 * v + r] = lam[r];
    }
}

__global__ void k_vx_emit(int64_t V, const int64_t *__restrict__ vstart, const uint64_t *__restrict__ ckey,
                          const int64_t *__restrict__ count, const double *__restrict__ s1,
                          const double *__restrict__ s2, CellLayout L, const int64_t *__restrict__ keep,
                          const int64_t *__restrict__ vrank, const int64_t *__restrict__ coff, int32_t level,
                          int64_t base_v, int64_t base_c, int32_t *__restrict__ o_vox, int32_t *__restrict__ o_scan,
                          int64_t *__restrict__ o_cnt, double *__restrict__ o_s1, double *__restrict__ o_s2,
                          int32_t *__restrict__ o_level, int32_t *__restrict__ o_cell) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V || !keep[v]) return;
    const int64_t a = vstart[v], b = vstart[v + 1];
    const int64_t vo = base_v + vrank[v];
    for (int64_t c = a; c < b; c++) {
        int64_t cc[3];
        int32_t s;
        vx_unpack(L, ckey[c], cc, s);
        const int64_t o = base_c + coff[v] + (c - a);
        o_vox[o] = (int32_t)vo;
        o_scan[o] = s;
        o_cnt[o] = count[c];
#pragma unroll
        for (int r = 0; r < 3; r++) o_s1[3 * o + r] = s1[3 * c + r];
#pragma unroll
        for (int r = 0; r < 6; r++) o_s2[6 * o + r] = s2[6 * c + r];
        if (c == a) {
            o_level[vo] = level;
#pragma unroll
            for (int r = 0; r < 3; r++) o_cell[3 * vo + r] = (int32_t)cc[r];
        }
    }
}

// cell and scan of each cluster, written out (batches of the host stream)
__global__ void k_vx_decode(int64_t C, const uint64_t *__restrict__ ckey, CellLayout L, int32_t *__restrict__ cell,
                            int32_t *__restrict__ cscan) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    int64_t cc[3];
    int32_t sc;
    vx_unpack(L, ckey[c], cc, sc);
#pragma unroll
    for (int r = 0; r < 3; r++) cell[3 * c + r] = (int32_t)cc[r];
    cscan[c] = sc;
}

// bounding box of explicit cluster cells (block partials in the layout of
// k_vx_cells, flags 0)
__global__ __launch_bounds__(VX_THREADS) void k_vx_cell_box(int64_t C, const int32_t *__restrict__ cell,
                                                            int32_t *__restrict__ bpart) {
    constexpr int NW = VX_THREADS / 64;
    __shared__ int red[NW];
    int lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, nhi[3] = {INT32_MAX, INT32_MAX, INT32_MAX};
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < C; c += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int r = 0; r < 3; r++) {
            lo[r] = min(lo[r], cell[3 * c + r]);
            nhi[r] = min(nhi[r], -cell[3 * c + r]);
        }
    }
    int *out = bpart + 7LL * blockIdx.x;
#pragma unroll
    for (int r = 0; r < 3; r++) {
        const int a = block_min_i<NW>(lo[r], red);
        const int b = block_min_i<NW>(nhi[r], red);
        if (threadIdx.x == 0) {
            out[r] = a;
            out[3 + r] = b;
        }
    }
    if (threadIdx.x == 0) out[6] = 0;
}

__global__ void k_vx_keys_cells(int64_t C, const int32_t *__restrict__ cell, const int32_t *__restrict__ cscan,
                                CellLayout L, uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C) return;
    keys[c] = vx_pack(L, cell[3 * c], cell[3 * c + 1], cell[3 * c + 2], cscan[c]);
    vals[c] = (uint32_t)c;
}

// one level's clusters (keys in (cell, scan) order) and its selection
struct VxLevel {
    CellLayout L;
    int64_t C = 0, V = 0, Vk = 0, Ck = 0;
    uint64_t *ckey = nullptr;
    int64_t *count = nullptr;
    double *s1 = nullptr, *s2 = nullptr;
    int64_t *vstart = nullptr, *keep = nullptr, *vrank = nullptr, *coff = nullptr;
};

// sort and scan buffers for up to cap entries
struct VxWork {
    uint64_t *keys = nullptr;
    uint32_t *vals = nullptr;
    int64_t *flags = nullptr, *total = nullptr;
    char *ws = nullptr;
    int64_t cap = 0;
};

}  // namespace ba

struct ba_voxel_map {
    ba::DevArena mem;
    int64_t n_points = 0, n_clusters = 0;
    int32_t n_voxels = 0, levels = 0, n_scans = 0, n_batches = 0;
    int64_t lv[BA_VOXEL_MAX_LEVELS][4] = {};
    int32_t *voxel = nullptr, *scan = nullptr, *vlevel = nullptr, *vcell = nullptr;
    int64_t *count = nullptr;
    double *sum = nullptr, *sumsq = nullptr;
};

namespace ba {

static ba_status sync_read(void *dst, const void *src, size_t bytes, hipStream_t s) {
    BA_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
    BA_HIP(hipStreamSynchronize(s));
    return BA_OK;
}

static ba_status work_alloc(DevArena &a, VxWork &w, int64_t cap) {
    w.cap = cap;
    BA_TRY(a.alloc(&w.keys, cap));
    BA_TRY(a.alloc(&w.vals, cap));
    BA_TRY(a.alloc(&w.flags, cap + 1));
    BA_TRY(a.alloc(&w.total, 1));
    BA_TRY(a.alloc(&w.ws, (int64_t)std::max(radix_sort_workspace_bytes(cap), scan_workspace_bytes(cap))));
    return BA_OK;
}

// segments of sorted keys that agree above bit `shift`: their number and
// their starts (length n_seg + 1)
static ba_status vx_segments(DevArena &tmp, VxWork &w, const uint64_t *keys, int64_t n, int shift,
                             int64_t **starts, int64_t *n_seg, hipStream_t s) {
    hipLaunchKernelGGL(k_vx_heads, dim3(vx_nblk(n)), dim3(VX_THREADS), 0, s, n, keys, shift, w.flags);
    BA_HIP(exclusive_scan_i64(w.flags, w.flags, n, w.total, w.ws, s));
    BA_TRY(sync_read(n_seg, w.total, sizeof(int64_t), s));
    BA_TRY(tmp.alloc(starts, *n_seg + 1));
    hipLaunchKernelGGL(k_vx_starts, dim3(vx_nblk(n)), dim3(VX_THREADS), 0, s, n, keys, shift, w.flags, *starts,
                       *n_seg);
    BA_HIP(hipGetLastError());
    return BA_OK;
}

static ba_status check_layout(const CellLayout &L) {
    if (L.total > 64) {
        set_error("cell range needs %d key bits (at most 64): use a larger d", L.total);
        return BA_E_UNSUPPORTED;
    }
    return BA_OK;
}

// Sort the m keys in w (layout cur.L) and form cur's clusters: raw sums of
// points (x non-null) or of the child clusters.
static ba_status vx_form_level(DevArena &tmp, VxWork &w, int64_t m, const double *x, const double *y,
                               const double *z, const int64_t *ccount, const double *cs1, const double *cs2,
                               VxLevel &cur, hipStream_t s) {
    BA_HIP(radix_sort_pairs(w.keys, w.vals, m, cur.L.total, w.ws, s));
    int64_t *starts;
    BA_TRY(vx_segments(tmp, w, w.keys, m, 0, &starts, &cur.C, s));
    BA_TRY(tmp.alloc(&cur.ckey, cur.C));
    BA_TRY(tmp.alloc(&cur.count, cur.C));
    BA_TRY(tmp.alloc(&cur.s1, 3 * cur.C));
    BA_TRY(tmp.alloc(&cur.s2, 6 * cur.C));
    if (x)
        hipLaunchKernelGGL(k_vx_sum_points, dim3(vx_nblk(cur.C * VX_SUM_LANES)), dim3(VX_THREADS), 0, s, cur.C, starts, w.keys, w.vals,
                           x, y, z, cur.ckey, cur.count, cur.s1, cur.s2);
    else
        hipLaunchKernelGGL(k_vx_sum_clusters, dim3(vx_nblk(cur.C)), dim3(VX_THREADS), 0, s, cur.C, starts, w.keys,
                           w.vals, ccount, cs1, cs2, cur.ckey, cur.count, cur.s1, cur.s2);
    BA_HIP(hipGetLastError());
    return BA_OK;
}

// World cells of n device points (asynchronous; box receives the bounding box
// and flags) and, after a wait, the layout from that box.
static ba_status vx_cells_launch(DevArena &tmp, const double *x, const double *y, const double *z,
                                 const int32_t *scan, int64_t n, int32_t n_scans, const double *poses, double d,
                                 int32_t *cell, int32_t **box, hipStream_t s) {
    int32_t *bpart;
    BA_TRY(tmp.alloc(&bpart, 7LL * VX_BOX_BLOCKS));
    BA_TRY(tmp.alloc(box, 7));
    const int nb = (int)std::min<int64_t>(VX_BOX_BLOCKS, vx_nblk(n));
    hipLaunchKernelGGL(k_vx_cells, dim3(nb), dim3(VX_THREADS), 0, s, n, x, y, z, scan, n_scans, poses, d, cell,
                       bpart);
    hipLaunchKernelGGL(k_vx_bbox, dim3(1), dim3(VX_THREADS), 0, s, nb, bpart, *box);
    BA_HIP(hipGetLastError());
    return BA_OK;
}

static ba_status vx_cells_layout(const int32_t *box, int32_t n_scans, CellLayout *L, hipStream_t s) {
    int32_t hb[7];
    BA_TRY(sync_read(hb, box, sizeof(hb), s));
    if (hb[6]) {
        set_error("invalid points (flags 0x%x: 1 non-finite world point, 2 scan out of range, 4 cell index beyond "
                  "2^30 at edge d)",
                  hb[6]);
        return BA_E_ARG;
    }
    int64_t lo[3] = {hb[0], hb[1], hb[2]}, hi[3] = {-(int64_t)hb[3], -(int64_t)hb[4], -(int64_t)hb[5]};
    *L = make_layout(lo, hi, n_scans);
    return check_layout(*L);
}

// Planarity decisions of one level and its kept counts.
static ba_status vx_select_level(DevArena &tmp, VxWork &w, VxLevel &cur, const double *poses,
                                 const ba_voxelize_options *opt, hipStream_t s) {
    // cells of this level: segments of the cluster keys without the scan bits
    BA_TRY(vx_segments(tmp, w, cur.ckey, cur.C, cur.L.sbits, &cur.vstart, &cur.V, s));
    BA_TRY(tmp.alloc(&cur.keep, cur.V + 1));
    BA_TRY(tmp.alloc(&cur.coff, cur.V + 1));
    BA_TRY(tmp.alloc(&cur.vrank, cur.V + 1));
    hipLaunchKernelGGL(k_vx_select, dim3(vx_nblk(cur.V)), dim3(VX_THREADS), 0, s, cur.V, cur.vstart, cur.ckey,
                       cur.count, cur.s1, cur.s2, cur.L, poses, opt->tau, opt->min_scans, cur.keep, cur.coff,
                       (double *)nullptr);
    BA_HIP(hipGetLastError());
    BA_HIP(exclusive_scan_i64(cur.keep, cur.vrank, cur.V, w.total, w.ws, s));
    BA_TRY(sync_read(&cur.Vk, w.total, sizeof(int64_t), s));
    BA_HIP(exclusive_scan_i64(cur.coff, cur.coff, cur.V, w.total, w.ws, s));
    BA_TRY(sync_read(&cur.Ck, w.total, sizeof(int64_t), s));
    return BA_OK;
}

// From the level-1 clusters in lv[0]: levels 2..L (Eq. 5), the selection of
// every level and the concatenated output.
static ba_status vx_finish(DevArena &tmp, VxWork &w, std::vector<VxLevel> &lv, int32_t n_scans,
                           const double *poses, const ba_voxelize_options *opt, ba_voxel_map *M, hipStream_t s) {
    const int levels = (int)lv.size();
    BA_TRY(vx_select_level(tmp, w, lv[0], poses, opt, s));
    for (int k = 1; k < levels; k++) {
        VxLevel &cur = lv[k];
        const VxLevel &prev = lv[k - 1];
        int64_t plo[3], phi[3];
        for (int r = 0; r < 3; r++) {
            plo[r] = prev.L.lo[r] >> 1;
            phi[r] = prev.L.hi[r] >> 1;
        }
        cur.L = make_layout(plo, phi, n_scans);
        hipLaunchKernelGGL(k_vx_keys_up, dim3(vx_nblk(prev.C)), dim3(VX_THREADS), 0, s, prev.C, prev.ckey, prev.L,
                           cur.L, w.keys, w.vals);
        BA_HIP(hipGetLastError());
        BA_TRY(vx_form_level(tmp, w, prev.C, nullptr, nullptr, nullptr, prev.count, prev.s1, prev.s2, cur, s));
        BA_TRY(vx_select_level(tmp, w, cur, poses, opt, s));
    }
    int64_t Vout = 0, Cout = 0;
    for (auto &l : lv) {
        Vout += l.Vk;
        Cout += l.Ck;
    }
    if (Vout > INT32_MAX) {
        set_error("%lld selected voxels exceed the int32 voxel ids", (long long)Vout);
        return BA_E_UNSUPPORTED;
    }
    BA_TRY(M->mem.alloc(&M->voxel, Cout));
    BA_TRY(M->mem.alloc(&M->scan, Cout));
    BA_TRY(M->mem.alloc(&M->count, Cout));
    BA_TRY(M->mem.alloc(&M->sum, 3 * Cout));
    BA_TRY(M->mem.alloc(&M->sumsq, 6 * Cout));
    BA_TRY(M->mem.alloc(&M->vlevel, Vout));
    BA_TRY(M->mem.alloc(&M->vcell, 3 * Vout));
    int64_t bv = 0, bc = 0;
    for (int k = 0; k < levels; k++) {
        VxLevel &l = lv[k];
        hipLaunchKernelGGL(k_vx_emit, dim3(vx_nblk(l.V)), dim3(VX_THREADS), 0, s, l.V, l.vstart, l.ckey, l.count,
                           l.s1, l.s2, l.L, l.keep, l.vrank, l.coff, k + 1, bv, bc, M->voxel, M->scan, M->count,
                           M->sum, M->sumsq, M->vlevel, M->vcell);
        BA_HIP(hipGetLastError());
        M->lv[k][0] = l.V;
        M->lv[k][1] = l.C;
        M->lv[k][2] = l.Vk;
        M->lv[k][3] = l.Ck;
        bv += l.Vk;
        bc += l.Ck;
    }
    BA_HIP(hipStreamSynchronize(s));
    M->n_clusters = Cout;
    M->n_voxels = (int32_t)Vout;
    M->levels = levels;
    M->n_scans = n_scans;
    return BA_OK;
}

static ba_status voxelize(const double *x, const double *y, const double *z, const int32_t *scan, int64_t n,
                          int32_t n_scans, const double *poses, const ba_voxelize_options *opt, ba_voxel_map *M,
                          hipStream_t s) {
    DevArena tmp;
    int32_t *cell;
    BA_TRY(tmp.alloc(&cell, 3 * n));
    std::vector<VxLevel> lv(opt->levels);
    int32_t *box;
    BA_TRY(vx_cells_launch(tmp, x, y, z, scan, n, n_scans, poses, opt->d, cell, &box, s));
    BA_TRY(vx_cells_layout(box, n_scans, &lv[0].L, s));
    VxWork w;
    BA_TRY(work_alloc(tmp, w, n));   // the points are the largest level
    hipLaunchKernelGGL(k_vx_keys_points, dim3(vx_nblk(n)), dim3(VX_THREADS), 0, s, n, cell, scan, lv[0].L, w.keys,
                       w.vals);
    BA_HIP(hipGetLastError());
    BA_TRY(vx_form_level(tmp, w, n, x, y, z, nullptr, nullptr, nullptr, lv[0], s));
    BA_TRY(vx_finish(tmp, w, lv, n_scans, poses, opt, M, s));
    M->n_points = n;
    return BA_OK;
}

// ---------------------------------------------------------------- host stream
// Copies of host memory by a few threads (pageable sources are staged into
// pinned buffers before their transfer).
static void parallel_copy(void *dst, const void *src, size_t bytes) {
    constexpr size_t CHUNK = (size_t)8 << 20;
    const int nt = (int)std::min<size_t>(8, (bytes + CHUNK - 1) / CHUNK);
    if (nt <= 1) {
        std::memcpy(dst, src, bytes);
        return;
    }
    std::vector<std::thread> th;
    const size_t per = (bytes + nt - 1) / nt;
    for (int t = 0; t < nt; t++) {
        const size_t a = per * t, b = std::min(bytes, a + per);
        if (a >= b) break;
        th.emplace_back([=] { std::memcpy((char *)dst + a, (const char *)src + a, b - a); });
    }
    for (auto &t : th) t.join();
}

static bool host_pinned(const void *p) {
    hipPointerAttribute_t at;
    hipError_t e = hipPointerGetAttributes(&at, p);
    (void)hipGetLastError();
    return e == hipSuccess && at.type == hipMemoryTypeHost;
}

// one batch's level-1 clusters with their cells written out
struct VxBatch {
    int64_t C = 0;
    int32_t *cell = nullptr, *scan = nullptr;
    int64_t *count = nullptr;
    double *s1 = nullptr, *s2 = nullptr;
};

struct HostStream {
    hipStream_t copy = nullptr;
    hipEvent_t copied[2] = {nullptr, nullptr}, consumed[2] = {nullptr, nullptr};
    void *pinned[2] = {nullptr, nullptr};
    ~HostStream() {
        if (copy) (void)hipStreamSynchronize(copy);
        for (int k = 0; k < 2; k++) {
            if (copied[k]) (void)hipEventSynchronize(copied[k]);
            if (consumed[k]) (void)hipEventSynchronize(consumed[k]);
        }
        for (int k = 0; k < 2; k++) {
            if (pinned[k]) (void)hipHostFree(pinned[k]);
            if (copied[k]) (void)hipEventDestroy(copied[k]);
            if (consumed[k]) (void)hipEventDestroy(consumed[k]);
        }
        if (copy) (void)hipStreamDestroy(copy);
    }
};

static ba_status voxelize_host(const double *hx, const double *hy, const double *hz, const int32_t *hscan,
                               int64_t n, int32_t n_scans, const double *poses, const ba_voxelize_options *opt,
                               const ba_stream_options *so, ba_voxel_map *M, hipStream_t s) {
    constexpr int64_t WORK_BYTES = 2 * 28 + 12 + 8 + 4 + 8 + 12 + 16;   // per batch point: buffers, cells, sort
    int64_t B = so ? so->batch_points : 0;
    if (B <= 0) {
        size_t fr = 0, tot = 0;
        BA_HIP(hipMemGetInfo(&fr, &tot));
        const double alpha = (so && so->alpha > 0.0) ? so->alpha : 0.5;
        B = (int64_t)(alpha * (double)fr / (double)WORK_BYTES);
    }
    B = std::max<int64_t>(1024, std::min<int64_t>(B, n));
    const bool pinned_in = host_pinned(hx) && host_pinned(hy) && host_pinned(hz) && host_pinned(hscan);
    HostStream hs;
    BA_HIP(hipStreamCreateWithFlags(&hs.copy, hipStreamNonBlocking));
    for (int k = 0; k < 2; k++) {
        BA_HIP(hipEventCreateWithFlags(&hs.copied[k], hipEventDisableTiming));
        BA_HIP(hipEventCreateWithFlags(&hs.consumed[k], hipEventDisableTiming));
        if (!pinned_in) BA_HIP(hipHostMalloc(&hs.pinned[k], (size_t)B * 28, hipHostMallocDefault));
    }
    DevArena tmp;
    double *dx[2], *dy[2], *dz[2];
    int32_t *ds[2], *cell;
    for (int k = 0; k < 2; k++) {
        BA_TRY(tmp.alloc(&dx[k], B));
        BA_TRY(tmp.alloc(&dy[k], B));
        BA_TRY(tmp.alloc(&dz[k], B));
        BA_TRY(tmp.alloc(&ds[k], B));
    }
    BA_TRY(tmp.alloc(&cell, 3 * B));
    VxWork w;
    BA_TRY(work_alloc(tmp, w, B));
    const int64_t nbat = (n + B - 1) / B;
    std::vector<VxBatch> bat(nbat);
    // stage batch b into pinned buffer b % 2 (pageable input) and start its transfer
    auto start_copy = [&](int64_t b) -> ba_status {
        const int k = (int)(b & 1);
        const int64_t a = b * B, m = std::min(B, n - a);
        const double *sx = hx + a, *sy = hy + a, *sz = hz + a;
        const int32_t *ss = hscan + a;
        if (!pinned_in) {
            BA_HIP(hipEventSynchronize(hs.copied[k]));   // the buffer's previous transfer has finished
            char *pb = (char *)hs.pinned[k];
            parallel_copy(pb, sx, (size_t)m * 8);
            parallel_copy(pb + (size_t)B * 8, sy, (size_t)m * 8);
            parallel_copy(pb + (size_t)B * 16, sz, (size_t)m * 8);
            parallel_copy(pb + (size_t)B * 24, ss, (size_t)m * 4);
            sx = (const double *)pb;
            sy = (const double *)(pb + (size_t)B * 8);
            sz = (const double *)(pb + (size_t)B * 16);
            ss = (const int32_t *)(pb + (size_t)B * 24);
        }
        // the device buffer k is free once batch b - 2 has been clustered
        BA_HIP(hipStreamWaitEvent(hs.copy, hs.consumed[k], 0));
        BA_HIP(hipMemcpyAsync(dx[k], sx, (size_t)m * 8, hipMemcpyHostToDevice, hs.copy));
        BA_HIP(hipMemcpyAsync(dy[k], sy, (size_t)m * 8, hipMemcpyHostToDevice, hs.copy));
        BA_HIP(hipMemcpyAsync(dz[k], sz, (size_t)m * 8, hipMemcpyHostToDevice, hs.copy));
        BA_HIP(hipMemcpyAsync(ds[k], ss, (size_t)m * 4, hipMemcpyHostToDevice, hs.copy));
        BA_HIP(hipEventRecord(hs.copied[k], hs.copy));
        return BA_OK;
    };
    BA_TRY(start_copy(0));
    for (int64_t b = 0; b < nbat; b++) {
        const int k = (int)(b & 1);
        const int64_t m = std::min(B, n - b * B);
        BA_HIP(hipStreamWaitEvent(s, hs.copied[k], 0));
        VxLevel l1;
        int32_t *box;
        BA_TRY(vx_cells_launch(tmp, dx[k], dy[k], dz[k], ds[k], m, n_scans, poses, opt->d, cell, &box, s));
        // the next batch is staged and its transfer queued while this one is clustered
        if (b + 1 < nbat) BA_TRY(start_copy(b + 1));
        BA_TRY(vx_cells_layout(box, n_scans, &l1.L, s));
        hipLaunchKernelGGL(k_vx_keys_points, dim3(vx_nblk(m)), dim3(VX_THREADS), 0, s, m, cell, ds[k], l1.L, w.keys,
                           w.vals);
        BA_HIP(hipGetLastError());
        BA_TRY(vx_form_level(tmp, w, m, dx[k], dy[k], dz[k], nullptr, nullptr, nullptr, l1, s));
        VxBatch &o = bat[b];
        o.C = l1.C;
        BA_TRY(tmp.alloc(&o.cell, 3 * o.C));
        BA_TRY(tmp.alloc(&o.scan, o.C));
        o.count = l1.count;
        o.s1 = l1.s1;
        o.s2 = l1.s2;
        hipLaunchKernelGGL(k_vx_decode, dim3(vx_nblk(o.C)), dim3(VX_THREADS), 0, s, o.C, l1.ckey, l1.L, o.cell,
                           o.scan);
        BA_HIP(hipGetLastError());
        BA_HIP(hipEventRecord(hs.consumed[k], s));
    }
    // merge the batches' clusters of equal (cell, scan): one sort, raw sums added
    int64_t C = 0;
    for (auto &o : bat) C += o.C;
    int32_t *acell, *ascan;
    int64_t *acount;
    double *as1, *as2;
    BA_TRY(tmp.alloc(&acell, 3 * C));
    BA_TRY(tmp.alloc(&ascan, C));
    BA_TRY(tmp.alloc(&acount, C));
    BA_TRY(tmp.alloc(&as1, 3 * C));
    BA_TRY(tmp.alloc(&as2, 6 * C));
    int64_t off = 0;
    for (auto &o : bat) {
        BA_HIP(hipMemcpyAsync(acell + 3 * off, o.cell, (size_t)o.C * 12, hipMemcpyDeviceToDevice, s));
        BA_HIP(hipMemcpyAsync(ascan + off, o.scan, (size_t)o.C * 4, hipMemcpyDeviceToDevice, s));
        BA_HIP(hipMemcpyAsync(acount + off, o.count, (size_t)o.C * 8, hipMemcpyDeviceToDevice, s));
        BA_HIP(hipMemcpyAsync(as1 + 3 * off, o.s1, (size_t)o.C * 24, hipMemcpyDeviceToDevice, s));
        BA_HIP(hipMemcpyAsync(as2 + 6 * off, o.s2, (size_t)o.C * 48, hipMemcpyDeviceToDevice, s));
        off += o.C;
    }
    int32_t *bpart, *box;
    BA_TRY(tmp.alloc(&bpart, 7LL * VX_BOX_BLOCKS));
    BA_TRY(tmp.alloc(&box, 7));
    const int nb = (int)std::min<int64_t>(VX_BOX_BLOCKS, vx_nblk(C));
    hipLaunchKernelGGL(k_vx_cell_box, dim3(nb), dim3(VX_THREADS), 0, s, C, acell, bpart);
    hipLaunchKernelGGL(k_vx_bbox, dim3(1), dim3(VX_THREADS), 0, s, nb, bpart, box);
    BA_HIP(hipGetLastError());
    int32_t hb[7];
    BA_TRY(sync_read(hb, box, sizeof(hb), s));
    std::vector<VxLevel> lv(opt->levels);
    int64_t lo[3] = {hb[0], hb[1], hb[2]}, hi[3] = {-(int64_t)hb[3], -(int64_t)hb[4], -(int64_t)hb[5]};
    lv[0].L = make_layout(lo, hi, n_scans);
    BA_TRY(check_layout(lv[0].L));
    VxWork wm;
    BA_TRY(work_alloc(tmp, wm, C));
    hipLaunchKernelGGL(k_vx_keys_cells, dim3(vx_nblk(C)), dim3(VX_THREADS), 0, s, C, acell, ascan, lv[0].L, wm.keys,
                       wm.vals);
    BA_HIP(hipGetLastError());
    BA_TRY(vx_form_level(tmp, wm, C, nullptr, nullptr, nullptr, acount, as1, as2, lv[0], s));
    BA_TRY(vx_finish(tmp, wm, lv, n_scans, poses, opt, M, s));
    M->n_points = n;
    M->n_batches = (int32_t)nbat;
    return BA_OK;
}

}  // namespace ba

using namespace ba;

extern "C" {

static ba_status check_voxelize_args(const void *x, const void *y, const void *z, const void *scan, int64_t n,
                                     int32_t n_scans, const void *poses, const ba_voxelize_options *opt,
                                     ba_voxel_map **out) {
    if (!out) {
        set_error("out is null");
        return BA_E_ARG;
    }
    *out = nullptr;
    if (!x || !y || !z || !scan || !poses || !opt) {
        set_error("null argument");
        return BA_E_ARG;
    }
    if (n < 1 || n > (int64_t)0xFFFFFFFF || n_scans < 1) {
        set_error("point count %lld out of [1, 2^32) or no scans", (long long)n);
        return BA_E_ARG;
    }
    if (!(opt->d > 0.0) || !std::isfinite(opt->d) || !(opt->tau > 0.0) || !std::isfinite(opt->tau) ||
        opt->levels < 1 || opt->levels > BA_VOXEL_MAX_LEVELS || opt->min_scans < 0) {
        set_error("voxelize options out of range (d %g, levels %d, tau %g, min_scans %d)", opt->d, opt->levels,
                  opt->tau, opt->min_scans);
        return BA_E_ARG;
    }
    return BA_OK;
}

ba_status ba_voxelize(const double *x, const double *y, const double *z, const int32_t *scan, int64_t n,
                      int32_t n_scans, const double *poses, const ba_voxelize_options *opt, ba_voxel_map **out,
                      hipStream_t stream) {
    BA_TRY(check_voxelize_args(x, y, z, scan, n, n_scans, poses, opt, out));
    ba_voxel_map *M = new ba_voxel_map();
    ba_status st = voxelize(x, y, z, scan, n, n_scans, poses, opt, M, stream);
    if (st != BA_OK) {
        (void)hipStreamSynchronize(stream);
        delete M;
        return st;
    }
    *out = M;
    return BA_OK;
}

ba_status ba_voxelize_host(const double *x, const double *y, const double *z, const int32_t *scan, int64_t n,
                           int32_t n_scans, const double *poses, const ba_voxelize_options *opt,
                           const ba_stream_options *so, ba_voxel_map **out, hipStream_t stream) {
    BA_TRY(check_voxelize_args(x, y, z, scan, n, n_scans, poses, opt, out));
    if (so && (so->alpha < 0.0 || so->alpha > 1.0 || !std::isfinite(so->alpha) || so->batch_points < 0)) {
        set_error("stream options out of range (alpha %g, batch_points %lld)", so->alpha,
                  (long long)so->batch_points);
        return BA_E_ARG;
    }
    ba_voxel_map *M = new ba_voxel_map();
    ba_status st = voxelize_host(x, y, z, scan, n, n_scans, poses, opt, so, M, stream);
    if (st != BA_OK) {
        (void)hipStreamSynchronize(stream);
        delete M;
        return st;
    }
    *out = M;
    return BA_OK;
}

ba_status ba_voxel_map_get_info(const ba_voxel_map *m, ba_voxel_map_info *info) {
    if (!m || !info) {
        set_error("null argument");
        return BA_E_ARG;
    }
    std::memset(info, 0, sizeof(*info));
    info->n_points = m->n_points;
    info->n_clusters = m->n_clusters;
    info->n_voxels = m->n_voxels;
    info->levels = m->levels;
    info->n_scans = m->n_scans;
    info->n_batches = m->n_batches;
    for (int k = 0; k < m->levels; k++) {
        info->level_voxels[k] = m->lv[k][0];
        info->level_clusters[k] = m->lv[k][1];
        info->level_kept_voxels[k] = m->lv[k][2];
        info->level_kept_clusters[k] = m->lv[k][3];
    }
    info->device_bytes = (int64_t)m->mem.bytes;
    return BA_OK;
}

ba_status ba_voxel_map_export(const ba_voxel_map *m, int32_t *voxel, int32_t *scan, int64_t *count, double *sum,
                              double *sumsq, int32_t *voxel_level, int32_t *voxel_cell, hipStream_t stream) {
    if (!m) {
        set_error("null map");
        return BA_E_ARG;
    }
    const size_t C = (size_t)m->n_clusters, V = (size_t)m->n_voxels;
    auto cp = [&](void *dst, const void *src, size_t bytes) -> ba_status {
        if (dst && bytes) BA_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, stream));
        return BA_OK;
    };
    BA_TRY(cp(voxel, m->voxel, C * sizeof(int32_t)));
    BA_TRY(cp(scan, m->scan, C * sizeof(int32_t)));
    BA_TRY(cp(count, m->count, C * sizeof(int64_t)));
    BA_TRY(cp(sum, m->sum, 3 * C * sizeof(double)));
    BA_TRY(cp(sumsq, m->sumsq, 6 * C * sizeof(double)));
    BA_TRY(cp(voxel_level, m->vlevel, V * sizeof(int32_t)));
    BA_TRY(cp(voxel_cell, m->vcell, 3 * V * sizeof(int32_t)));
    return BA_OK;
}

ba_status ba_voxel_map_destroy(ba_voxel_map *m) {
    if (!m) return BA_OK;
    (void)hipDeviceSynchronize();
    delete m;
    return BA_OK;
}

}  // extern "C"
