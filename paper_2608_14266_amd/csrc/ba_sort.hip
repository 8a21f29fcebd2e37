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

// per-thread digit counts into cnt[d][t]
__device__ __forceinline__ void tile_counts(const uint64_t *__restrict__ keys, int64_t n, int shift,
                                            uint32_t (*cnt)[RS_THREADS]) {
    int t = threadIdx.x;
#pragma unroll
    for (int d = 0; d < RS_BINS; d++) cnt[d][t] = 0;
    int64_t base = (int64_t)blockIdx.x * RS_TILE + (int64_t)t * RS_IPT;
    for (int k = 0; k < RS_IPT; k++) {
        int64_t i = base + k;
        if (i < n) cnt[digit_of(keys[i], shift)][t]++;
    }
}

__global__ __launch_bounds__(RS_THREADS) void k_radix_hist(const uint64_t *__restrict__ keys, int64_t n, int shift,
                                                           int64_t *__restrict__ hist, int64_t nblocks) {
    __shared__ uint32_t cnt[RS_BINS][RS_THREADS];
    tile_counts(keys, n, shift, cnt);
    __syncthreads();
    // 16 bins x 256 threads: wave w sums bins 4w..4w+3
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int d = 4 * w; d < 4 * w + 4; d++) {
        uint32_t s = cnt[d][lane] + cnt[d][lane + 64] + cnt[d][lane + 128] + cnt[d][lane + 192];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (lane == 0) hist[(int64_t)d * nblocks + blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(RS_THREADS) void k_radix_scatter(const uint64_t *__restrict__ keys_in,
                                                              const uint32_t *__restrict__ vals_in, int64_t n,
                                                              int shift, const int64_t *__restrict__ gofs,
                                                              int64_t nblocks, uint64_t *__restrict__ keys_out,
                                                              uint32_t *__restrict__ vals_out) {
    __shared__ uint32_t cnt[RS_BINS][RS_THREADS];
    __shared__ int64_t lw[RS_THREADS / 64];
    __shared__ uint32_t tstart[RS_BINS];
    __shared__ int64_t gbase[RS_BINS];
    int t = threadIdx.x;
    tile_counts(keys_in, n, shift, cnt);
    if (t < RS_BINS) gbase[t] = gofs[(int64_t)t * nblocks + blockIdx.x];
    __syncthreads();
    // 2-D exclusive scan over flattened (d, t): thread k owns entries [16k, 16k+16)
    uint32_t *flat = &cnt[0][0];
    uint32_t loc[16];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < 16; k++) {
        loc[k] = flat[16 * t + k];
        s += loc[k];
    }
    int64_t tot;
    int64_t ex = block_excl_scan((int64_t)s, lw, tot);
    uint32_t run = (uint32_t)ex;
#pragma unroll
    for (int k = 0; k < 16; k++) {
        flat[16 * t + k] = run;
        run += loc[k];
    }
    __syncthreads();
    if (t < RS_BINS) tstart[t] = cnt[t][0];
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * RS_TILE + (int64_t)t * RS_IPT;
    for (int k = 0; k < RS_IPT; k++) {
        int64_t i = base + k;
        if (i < n) {
            uint64_t key = keys_in[i];
            int d = digit_of(key, shift);
            uint32_t r = cnt[d][t]++;
            int64_t pos = gbase[d] + (int64_t)(r - tstart[d]);
            keys_out[pos] = key;
            vals_out[pos] = vals_in[i];
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
