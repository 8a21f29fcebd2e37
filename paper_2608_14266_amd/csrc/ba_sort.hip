// Device-wide primitives for the one-time problem build (paper Sec. IV-A,
// "Standard Primitives": sort_by_key, exclusive_scan, scatter):
//   * exclusive prefix scan of int64 (reduce-then-scan, three launches);
//   * stable LSD radix sort of (uint64 key, uint32 value) pairs with 8-bit
//     digits: per-tile digit histograms, a scan of the (digit, tile) counts
//     and a stable scatter whose within-tile ranks come from wave ballots
//     and per-wave digit counts, so equal keys keep their input order.
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
static constexpr int RS_WAVES = RS_THREADS / 64;
static constexpr int RS_IPT = 16;
static constexpr int RS_TILE = RS_THREADS * RS_IPT;
static constexpr int RS_BITS = 8;                 // bits per pass
static constexpr int RS_BINS = 1 << RS_BITS;      // one digit per thread of a block
static_assert(RS_BINS == RS_THREADS, "a block handles one digit per thread");

__device__ __forceinline__ int digit_of(uint64_t k, int shift) { return (int)((k >> shift) & (RS_BINS - 1)); }

// Lanes of the wave holding the same digit d (d == RS_BINS marks an empty
// slot): a ballot per bit of d, RS_BITS + 1 bits.
__device__ __forceinline__ uint64_t same_digit_lanes(int d) {
    uint64_t same = ~0ull;
#pragma unroll
    for (int b = 0; b <= RS_BITS; b++) {
        const bool bit = (d >> b) & 1;
        const uint64_t bal = __ballot(bit);
        same &= bit ? bal : ~bal;
    }
    return same;
}

// Tiles of RS_TILE keys; thread t of a block handles the items
// tile + 256 k + t (k = 0..15), so every load row is coalesced.  Per row, the
// first lane of each digit group adds the group's size to its wave's count of
// that digit (no two lanes of a wave add to one count).
__global__ __launch_bounds__(RS_THREADS) void k_radix_hist(const uint64_t *__restrict__ keys, int64_t n, int shift,
                                                           int64_t *__restrict__ hist, int64_t nblocks) {
    __shared__ uint32_t cnt[RS_WAVES][RS_BINS];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int v = 0; v < RS_WAVES; v++) cnt[v][t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE + t;
#pragma unroll 4
    for (int k = 0; k < RS_IPT; k++) {
        const int64_t i = base + (int64_t)k * RS_THREADS;
        const int d = i < n ? digit_of(keys[i], shift) : RS_BINS;
        const uint64_t same = same_digit_lanes(d);
        if (d < RS_BINS && (same & lt_mask) == 0) cnt[w][d] += (uint32_t)__popcll(same);
    }
    __syncthreads();
    uint32_t s = 0;
#pragma unroll
    for (int v = 0; v < RS_WAVES; v++) s += cnt[v][t];
    hist[(int64_t)t * nblocks + blockIdx.x] = s;
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
    __shared__ uint32_t wcnt[RS_WAVES][RS_BINS];
    __shared__ uint32_t run[RS_BINS];
    __shared__ uint32_t dstart[RS_BINS];
    __shared__ uint32_t wsum[RS_WAVES];
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
    run[t] = 0;
    gbase[t] = gofs[(int64_t)t * nblocks + blockIdx.x];
#pragma unroll
    for (int k = 0; k < RS_IPT; k++) {
#pragma unroll
        for (int v = 0; v < RS_WAVES; v++) wcnt[v][t] = 0;
        __syncthreads();
        const int d = dg[k];
        const uint64_t same = same_digit_lanes(d);
        const uint32_t rw = (uint32_t)__popcll(same & lt_mask);
        if (rw == 0 && d < RS_BINS) wcnt[w][d] = (uint32_t)__popcll(same);
        __syncthreads();
        if (d < RS_BINS) {
            uint32_t off = run[d];
            for (int v = 0; v < w; v++) off += wcnt[v][d];
            rank[k] = off + rw;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int v = 0; v < RS_WAVES; v++) add += wcnt[v][t];
        run[t] += add;
    }
    __syncthreads();
    // dstart = exclusive scan of run over the digits (thread t holds digit t)
    {
        const uint32_t r = run[t];
        uint32_t inc = r;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(inc, o, 64);
            if (lane >= o) inc += y;
        }
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        uint32_t before = 0;
        for (int v = 0; v < w; v++) before += wsum[v];
        dstart[t] = before + inc - r;
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
    const int passes = (bits + RS_BITS - 1) / RS_BITS;
    for (int pass = 0; pass < passes; pass++) {
        const int shift = RS_BITS * pass;
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
