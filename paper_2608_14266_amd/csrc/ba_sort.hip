// Device-wide primitives for the one-time problem build (paper Sec. IV-A,
// "Standard Primitives": sort_by_key, exclusive_scan, scatter):
//   * exclusive prefix scan of int64 (reduce-then-scan, three launches);
//   * stable LSD radix sort of (uint64 key, uint32 value) pairs with 4-bit
//     digits: per-tile digit histograms, a scan of the (digit, tile) counts
//     and a stable scatter whose within-tile ranks come from a 2-D scan over
//     (digit, thread) in LDS, so equal keys keep their input order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ba_internal.hpp"

namespace ba {

// ---------------------------------------------------------------- scan
static constexpr int SCAN_THREADS = 256;
static constexpr int SCAN_IPT = 8;
static constexpr int SCAN_TILE = SCAN_THREADS * SCAN_IPT;

__device__ __forceinline__ int64_t wave_incl_scan(int64_t v) {
    int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int64_t y = __shfl_up(v, o, 64);
        if (lane >= o) v += y;
    }
    return v;
}

// exclusive scan of one value per thread across a 256-thread block
__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t *lds_waves, int64_t &total) {
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t inc = wave_incl_scan(v);
    if (lane == 63) lds_waves[w] = inc;
    __syncthreads();
    int64_t base = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < SCAN_THREADS / 64; k++) {
        int64_t s = lds_waves[k];
        if (k < w) base += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return base + inc - v;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_reduce(const int64_t *__restrict__ in, int64_t n,
                                                              int64_t *__restrict__ bsum) {
    __shared__ int64_t lw[SCAN_THREADS / 64];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IPT;
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_IPT; k++)
        if (base + k < n) s += in[base + k];
    int64_t tot;
    block_excl_scan(s, lw, tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// single block: exclusive scan of nb block sums, writes total to *total
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_top(int64_t *__restrict__ bsum, int64_t nb,
                                                           int64_t *__restrict__ total) {
    __shared__ int64_t lw[SCAN_THREADS / 64];
    int64_t carry = 0;
    for (int64_t c0 = 0; c0 < nb; c0 += SCAN_TILE) {
        int64_t base = c0 + (int64_t)threadIdx.x * SCAN_IPT;
        int64_t v[SCAN_IPT];
        int64_t s = 0;
#pragma unroll
        for (int k = 0; k < SCAN_IPT; k++) {
            v[k] = (base + k < nb) ? bsum[base + k] : 0;
            s += v[k];
        }
        int64_t tot;
        int64_t ex = block_excl_scan(s, lw, tot);
        int64_t run = carry + ex;
#pragma unroll
        for (int k = 0; k < SCAN_IPT; k++) {
            if (base + k < nb) bsum[base + k] = run;
            run += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_down(const int64_t *__restrict__ in, int64_t n,
                                                            const int64_t *__restrict__ boff,
                                                            int64_t *__restrict__ out) {
    __shared__ int64_t lw[SCAN_THREADS / 64];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IPT;
    int64_t v[SCAN_IPT];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_IPT; k++) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    int64_t tot;
    int64_t run = boff[blockIdx.x] + block_excl_scan(s, lw, tot);
#pragma unroll
    for (int k = 0; k < SCAN_IPT; k++) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
}

size_t scan_workspace_bytes(int64_t n) {
    int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    return (size_t)(nb + 1) * sizeof(int64_t);
}

// out may alias in.  total (device pointer, may be null) receives the sum.
hipError_t exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *total, void *ws,
                              hipStream_t s) {
    int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    int64_t *bsum = (int64_t *)ws;
    if (n == 0) {
        if (total) return hipMemsetAsync(total, 0, sizeof(int64_t), s);
        return hipSuccess;
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, in, n, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_THREADS), 0, s, bsum, nb, total);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(SCAN_THREADS), 0, s, in, n, bsum, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- radix sort
static constexpr int RS_THREADS = 256;
static constexpr int RS_IPT = 16;
static constexpr int RS_TILE = RS_THREADS * RS_IPT;
static constexpr int RS_BINS = 16;

__device__ __forceinline__ int digit_of(uint64_t k, int shift) { return (int)((k >> shift) & (RS_BINS - 1)); }

// Tiles of RS_TILE keys; thread t of a block handles the items
// tile + 256 k + t (k = 0..15), so every load and store row is coalesced.
__global__ __launch_bounds__(RS_THREADS) void k_radix_hist(const uint64_t *__restrict__ keys, int64_t n, int shift,
                                                           int64_t *__restrict__ hist, int64_t nblocks) {
    __shared__ uint32_t cnt[RS_BINS][RS_THREADS];
    const int t = threadIdx.x;
#pragma unroll
    for (int d = 0; d < RS_BINS; d++) cnt[d][t] = 0;
    const int64_t base = (int64_t)blockIdx.x * RS_TILE + t;
#pragma unroll 4
    for (int k = 0; k < RS_IPT; k++) {
        const int64_t i = base + (int64_t)k * RS_THREADS;
        if (i < n) cnt[digit_of(keys[i], shift)][t]++;
    }
    __syncthreads();
    // 16 bins x 256 threads: wave w sums bins 4w..4w+3
    const int lane = t & 63, w = t >> 6;
    for (int d = 4 * w; d < 4 * w + 4; d++) {
        uint32_t s = cnt[d][lane] + cnt[d][lane + 64] + cnt[d][lane + 128] + cnt[d][lane + 192];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (lane == 0) hist[(int64_t)d * nblocks + blockIdx.x] = s;
    }
}

// Stable scatter of one tile: every item gets its rank among the tile's
// items of the same digit (rows in order; within a row, wave ballots give
// the rank among the wave's lanes and per-wave counts order the waves); the
// tile is then laid out by digit in LDS and written to the output as
// contiguous runs, one per digit.
__global__ __launch_bounds__(RS_THREADS) void k_radix_scatter(const uint64_t *__restrict__ keys_in,
                                                              const uint32_t *__restrict__ vals_in, int64_t n,
                                                              int shift, const int64_t *__restrict__ gofs,
                                                              int64_t nblocks, uint64_t *__restrict__ keys_out,
                                                              uint32_t *__restrict__ vals_out) {
    __shared__ uint64_t sk[RS_TILE];
    __shared__ uint32_t sv[RS_TILE];
    __shared__ uint32_t wcnt[RS_THREADS / 64][RS_BINS];
    __shared__ uint32_t run[RS_BINS];
    __shared__ uint32_t dstart[RS_BINS];
    __shared__ int64_t gbase[RS_BINS];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t tile0 = (int64_t)blockIdx.x * RS_TILE;
    const int tile_n = (int)(n - tile0 < RS_TILE ? n - tile0 : RS_TILE);
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint64_t key[RS_IPT];
    uint32_t val[RS_IPT];
    uint32_t rank[RS_IPT];
    int dg[RS_IPT];
#pragma unroll
    for (int k = 0; k < RS_IPT; k++) {
        const int64_t i = tile0 + (int64_t)k * RS_THREADS + t;
        const bool ok = i < n;
        key[k] = ok ? keys_in[i] : 0ull;
        val[k] = ok ? vals_in[i] : 0u;
        dg[k] = ok ? digit_of(key[k], shift) : RS_BINS;   // RS_BINS marks an empty slot
        rank[k] = 0;
    }
    if (t < RS_BINS) {
        run[t] = 0;
        gbase[t] = gofs[(int64_t)t * nblocks + blockIdx.x];
    }
#pragma unroll
    for (int k = 0; k < RS_IPT; k++) {
        if (t < (RS_THREADS / 64) * RS_BINS) wcnt[t / RS_BINS][t % RS_BINS] = 0;
        __syncthreads();
        const int d = dg[k];
        uint64_t same = ~0ull;
#pragma unroll
        for (int b = 0; b < 5; b++) {
            const bool bit = (d >> b) & 1;
            const uint64_t bal = __ballot(bit);
            same &= bit ? bal : ~bal;
        }
        const uint32_t rw = (uint32_t)__popcll(same & lt_mask);
        if (rw == 0 && d < RS_BINS) wcnt[w][d] = (uint32_t)__popcll(same);
        __syncthreads();
        if (d < RS_BINS) {
            uint32_t off = run[d];
            for (int v = 0; v < w; v++) off += wcnt[v][d];
            rank[k] = off + rw;
        }
        __syncthreads();
        if (t < RS_BINS) run[t] += wcnt[0][t] + wcnt[1][t] + wcnt[2][t] + wcnt[3][t];
    }
    __syncthreads();
    if (t == 0) {
        uint32_t a = 0;
        for (int d = 0; d < RS_BINS; d++) {
            dstart[d] = a;
            a += run[d];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < RS_IPT; k++) {
        if (dg[k] < RS_BINS) {
            const uint32_t p = dstart[dg[k]] + rank[k];
            if (p < (uint32_t)RS_TILE) {
                sk[p] = key[k];
                sv[p] = val[k];
            }
        }
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < RS_IPT; k++) {
        const int j = k * RS_THREADS + t;
        if (j < tile_n) {
            const uint64_t kk = sk[j];
            const int d = digit_of(kk, shift);
            const int64_t pos = gbase[d] + (int64_t)(j - (int)dstart[d]);
            if (pos >= 0 && pos < n) {
                keys_out[pos] = kk;
                vals_out[pos] = sv[j];
            }
        }
    }
}

size_t radix_sort_workspace_bytes(int64_t n) {
    int64_t nb = (n + RS_TILE - 1) / RS_TILE;
    size_t hist = (size_t)nb * RS_BINS * sizeof(int64_t);
    size_t alt = (size_t)n * (sizeof(uint64_t) + sizeof(uint32_t));
    return align_up(hist, 256) + align_up(scan_workspace_bytes(nb * RS_BINS), 256) + align_up(alt, 256) + 256;
}

// Sorts (keys, vals) in place by the low `bits` bits of the keys (stable).
hipError_t radix_sort_pairs(uint64_t *keys, uint32_t *vals, int64_t n, int bits, void *ws, hipStream_t s) {
    if (n <= 1 || bits <= 0) return hipSuccess;
    int64_t nb = (n + RS_TILE - 1) / RS_TILE;
    char *p = (char *)ws;
    int64_t *hist = (int64_t *)p;
    p += align_up((size_t)nb * RS_BINS * sizeof(int64_t), 256);
    void *scan_ws = p;
    p += align_up(scan_workspace_bytes(nb * RS_BINS), 256);
    uint64_t *k2 = (uint64_t *)p;
    uint32_t *v2 = (uint32_t *)(p + align_up((size_t)n * sizeof(uint64_t), 8));
    uint64_t *ka = keys, *kb = k2;
    uint32_t *va = vals, *vb = v2;
    int passes = (bits + 3) / 4;
    for (int pass = 0; pass < passes; pass++) {
        int shift = 4 * pass;
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(RS_THREADS), 0, s, ka, n, shift, hist, nb);
        hipError_t e = exclusive_scan_i64(hist, hist, nb * RS_BINS, nullptr, scan_ws, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(RS_THREADS), 0, s, ka, va, n, shift, hist, nb,
                           kb, vb);
        uint64_t *tk = ka; ka = kb; kb = tk;
        uint32_t *tv = va; va = vb; vb = tv;
    }
    if (ka != keys) {
        hipError_t e = hipMemcpyAsync(keys, ka, (size_t)n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(vals, va, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

}  // namespace ba
