// Device-wide exclusive scans and a stable LSD radix sort of (uint32 key,
// uint32 value) pairs, built from wavefront-level scans (shuffles) and
// ballot-based ranking.  No spin-waits: every scan is reduce-then-scan over
// two launches (the second sums the earlier tiles' totals itself), so every
// kernel finishes on its own.  Beyond kScanTile tiles (16.8M elements) the
// tiles' totals are themselves scanned first, recursively, and the second
// launch reads its tile's offset.
#include "common.hpp"

namespace apr {

namespace {

constexpr int kScanThreads = 1024;
constexpr int kScanItems = 4;                       // per thread
constexpr int kScanTile = kScanThreads * kScanItems;

template <class T>
__device__ inline T wave_incl_scan(T v)
{
    int lane = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        T t = __shfl_up(v, o, kWave);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive scan across a block of kScanThreads; returns the block total in *tot.
template <class T>
__device__ inline T block_excl_scan(T v, T *lds_waves, T *tot)
{
    int lane = lane_id(), w = threadIdx.x / kWave;
    constexpr int nw = kScanThreads / kWave;
    T incl = wave_incl_scan(v);
    if (lane == kWave - 1) lds_waves[w] = incl;
    __syncthreads();
    if (w == 0) {
        T s = lane < nw ? lds_waves[lane] : T(0);
        T si = wave_incl_scan(s);
        if (lane < nw) lds_waves[lane] = si - s;  // exclusive prefix of wave totals
        if (lane == nw - 1) lds_waves[nw] = si;
    }
    __syncthreads();
    T r = lds_waves[w] + incl - v;
    *tot = lds_waves[nw];
    __syncthreads();
    return r;
}

template <class T>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const T *in, int64_t n,
                                                               T *partial)
{
    __shared__ T lw[kScanThreads / kWave + 1];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) s += in[base + k];
    T tot;
    block_excl_scan(s, lw, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// Each tile: its offset is the sum of the earlier tiles' totals (summed here,
// nb <= kScanTile of them), then the tile's own exclusive scan; the last tile
// writes the grand total when asked.
template <class T>
__global__ __launch_bounds__(kScanThreads) void k_scan_down(const T *in, T *out, int64_t n,
                                                             const T *partial, T *total)
{
    __shared__ T lw[kScanThreads / kWave + 1];
    T pre = 0;
    for (int64_t k = threadIdx.x; k < (int64_t)blockIdx.x; k += kScanThreads) pre += partial[k];
    T off;
    block_excl_scan(pre, lw, &off);  // off: the block-wide sum of pre
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T v[kScanItems];
    T s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = base + k < n ? in[base + k] : T(0);
        s += v[k];
    }
    T tot;
    T ex = block_excl_scan(s, lw, &tot) + off;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = ex;
        ex += v[k];
    }
    if (total && threadIdx.x == 0 && blockIdx.x == gridDim.x - 1) *total = off + tot;
}

// The same with the tile's offset given: offset[blockIdx.x] is the sum of the
// earlier tiles' totals (an exclusive scan of them, for more tiles than one
// block can sum).
template <class T>
__global__ __launch_bounds__(kScanThreads) void k_scan_down_off(const T *in, T *out, int64_t n,
                                                                 const T *offset, T *total)
{
    __shared__ T lw[kScanThreads / kWave + 1];
    const T off = offset[blockIdx.x];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T v[kScanItems];
    T s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = base + k < n ? in[base + k] : T(0);
        s += v[k];
    }
    T tot;
    T ex = block_excl_scan(s, lw, &tot) + off;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = ex;
        ex += v[k];
    }
    if (total && threadIdx.x == 0 && blockIdx.x == gridDim.x - 1) *total = off + tot;
}

// level: recursion depth (each level has workspaces of its own)
template <class T>
int excl_scan(apr_ctx *c, const T *in, T *out, int64_t n, T *total_dev, const char *tag,
              int level = 0)
{
    if (n <= 0) {
        if (total_dev) {
            APR_HIP(c, hipMemsetAsync(total_dev, 0, sizeof(T), c->stream));
        }
        return APR_OK;
    }
    const int64_t nb = ceil_div(n, kScanTile);
    if (nb > ((int64_t)1 << 31)) return fail(c, APR_ERR_INVALID, "scan too long");
    const std::string nm = std::string(tag) + (level ? "_" + std::to_string(level) : "");
    T *partial = wsa<T>(c, nm.c_str(), (size_t)nb + 1);
    if (!partial) return fail(c, APR_ERR_HIP, "scan workspace");
    // one tile: no earlier tiles to sum (k_scan_down reads none of partial)
    if (nb > 1)
        hipLaunchKernelGGL(k_scan_reduce<T>, dim3((unsigned)nb), dim3(kScanThreads), 0,
                           c->stream, in, n, partial);
    if (nb <= kScanTile) {
        hipLaunchKernelGGL(k_scan_down<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, c->stream,
                           in, out, n, partial, total_dev);
    } else {
        // more tiles than one block sums: scan their totals first
        T *offset = wsa<T>(c, (nm + "_off").c_str(), (size_t)nb + 1);
        if (!offset) return fail(c, APR_ERR_HIP, "scan workspace");
        int rc = excl_scan<T>(c, partial, offset, nb, (T *)nullptr, tag, level + 1);
        if (rc) return rc;
        hipLaunchKernelGGL(k_scan_down_off<T>, dim3((unsigned)nb), dim3(kScanThreads), 0,
                           c->stream, in, out, n, offset, total_dev);
    }
    APR_LAUNCHED(c);
    return APR_OK;
}

// ------------------------------------------------------------------ radix sort
// 10-bit digits: the 30-bit Morton keys take three passes.
constexpr int kRadixBits = 10;
constexpr int kBins = 1 << kRadixBits;
constexpr int kSortThreads = 256;
constexpr int kBinsPerThread = kBins / kSortThreads;
// A block takes `rounds` rounds of 256 items (1 to 8): as many as keep about
// one block per CU busy, so that a small sort still spreads over the chip
// while a large one keeps its per-block histograms few.
constexpr int kMaxSortRounds = 8;
inline int sort_rounds(int64_t n)
{
    return (int)std::min<int64_t>(kMaxSortRounds, std::max<int64_t>(1, n / (kSortThreads * 256)));
}

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint32_t *keys, int64_t n,
                                                             int shift, uint32_t *hist,
                                                             int64_t nblocks, int rounds)
{
    __shared__ uint32_t h[kBins];
#pragma unroll
    for (int k = 0; k < kBinsPerThread; ++k) h[threadIdx.x + k * kSortThreads] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kSortThreads * rounds;
    for (int r = 0; r < rounds; ++r) {
        int64_t i = base + r * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & (kBins - 1)], 1u);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kBinsPerThread; ++k) {
        int b = threadIdx.x + k * kSortThreads;
        hist[(int64_t)b * nblocks + blockIdx.x] = h[b];
    }
}

// Stable scatter: in each round of 256 consecutive items, an item's rank among
// equal digits is (items of that digit in earlier rounds) + (in lower waves of
// this round) + (in lower lanes of its wave, from the ballot-built peer mask).
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout, int64_t n,
    int shift, const uint32_t *offs, int64_t nblocks, int rounds)
{
    constexpr int nw = kSortThreads / kWave;
    __shared__ uint32_t run[kBins];
    __shared__ uint32_t wc[nw][kBins];
#pragma unroll
    for (int k = 0; k < kBinsPerThread; ++k) {
        int b = threadIdx.x + k * kSortThreads;
        run[b] = offs[(int64_t)b * nblocks + blockIdx.x];
        for (int w = 0; w < nw; ++w) wc[w][b] = 0;
    }
    __syncthreads();
    int w = threadIdx.x / kWave;
    int64_t base = (int64_t)blockIdx.x * kSortThreads * rounds;
    for (int r = 0; r < rounds; ++r) {
        int64_t i = base + r * kSortThreads + threadIdx.x;
        bool valid = i < n;
        uint32_t key = valid ? kin[i] : 0u;
        uint32_t val = valid ? vin[i] : 0u;
        uint32_t d = (key >> shift) & (kBins - 1);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            bool bit = (d >> b) & 1u;
            uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        uint32_t rank = (uint32_t)__popcll(peers & lanemask_lt());
        bool leader = valid && (peers & lanemask_lt()) == 0;
        if (leader) wc[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = run[d] + rank;
            for (int v = 0; v < w; ++v) pos += wc[v][d];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kBinsPerThread; ++k) {
            int b = threadIdx.x + k * kSortThreads;
            uint32_t add = 0;
            for (int v = 0; v < nw; ++v) {
                add += wc[v][b];
                wc[v][b] = 0;
            }
            run[b] += add;
        }
        __syncthreads();
    }
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

int exclusive_scan_u32(apr_ctx *c, const uint32_t *in, uint32_t *out, int64_t n,
                       uint32_t *total_dev)
{
    return excl_scan<uint32_t>(c, in, out, n, total_dev, "scan_u32");
}

int exclusive_scan_i64(apr_ctx *c, const int64_t *in, int64_t *out, int64_t n,
                       int64_t *total_dev)
{
    return excl_scan<int64_t>(c, in, out, n, total_dev, "scan_i64");
}

int fill_i32(apr_ctx *c, int32_t *p, int32_t v, int64_t n)
{
    if (n <= 0) return APR_OK;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, c->stream,
                       p, v, n);
    APR_LAUNCHED(c);
    return APR_OK;
}

int fill_u32(apr_ctx *c, uint32_t *p, uint32_t v, int64_t n)
{
    if (n <= 0) return APR_OK;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, c->stream,
                       p, v, n);
    APR_LAUNCHED(c);
    return APR_OK;
}

// Sorts keys (low `bits` bits significant) and carries vals (callers pass a
// buffer).  The result is left in keys / vals, or, when keys_out and vals_out
// are given, wherever the last pass wrote it (no copy back): *keys_out and
// *vals_out point there (keys / vals, or the sort's own workspace).
int radix_sort_u32(apr_ctx *c, uint32_t *keys, uint32_t *vals, int64_t n, int bits,
                   uint32_t **keys_out, uint32_t **vals_out)
{
    if (keys_out) *keys_out = keys;
    if (vals_out) *vals_out = vals;
    if (n <= 1) return APR_OK;
    if (n >= (int64_t)1 << 31) return fail(c, APR_ERR_INVALID, "too many particles to sort");
    const int rounds = sort_rounds(n);
    int64_t nb = ceil_div(n, (int64_t)kSortThreads * rounds);
    uint32_t *k2 = wsa<uint32_t>(c, "sort_k2", (size_t)n);
    uint32_t *v2 = wsa<uint32_t>(c, "sort_v2", (size_t)n);
    uint32_t *hist = wsa<uint32_t>(c, "sort_hist", (size_t)(kBins * nb));
    if (!k2 || !v2 || !hist) return fail(c, APR_ERR_HIP, "sort workspace");
    int passes = (bits + kRadixBits - 1) / kRadixBits;
    uint32_t *ka = keys, *va = vals, *kb = k2, *vb = v2;
    for (int ps = 0; ps < passes; ++ps) {
        int shift = ps * kRadixBits;
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(kSortThreads), 0, c->stream,
                           ka, n, shift, hist, nb, rounds);
        APR_LAUNCHED(c);
        int rc = exclusive_scan_u32(c, hist, hist, kBins * nb, nullptr);
        if (rc) return rc;
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(kSortThreads), 0,
                           c->stream, ka, va, kb, vb, n, shift, hist, nb, rounds);
        APR_LAUNCHED(c);
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (keys_out && vals_out) {
        *keys_out = ka;
        *vals_out = va;
    } else if (ka != keys) {
        APR_HIP(c, hipMemcpyAsync(keys, ka, (size_t)n * 4, hipMemcpyDeviceToDevice, c->stream));
        APR_HIP(c, hipMemcpyAsync(vals, va, (size_t)n * 4, hipMemcpyDeviceToDevice, c->stream));
    }
    return APR_OK;
}

}  // namespace apr
