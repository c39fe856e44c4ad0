// Cell build: Morton keys -> stable radix sort -> in-place permutation of the
// particle state -> leaf cells of at most 64 consecutive particles -> a
// 64-ary tree of bounding boxes over the cells.
//
// Cells are cut from the leaves of the octree that the sorted keys define:
// a leaf is the largest Morton cube holding at most kLeafCap particles (and
// no larger than a segment: level 2 for periodic boxes, so a cell spans at
// most a quarter of the box per axis; 3 otherwise), and each leaf is cut
// into runs of 64.  Cubes keep the cells compact where the Morton curve
// jumps, e.g. across the thin layers of a disc.  The cell count is read back
// once per build so that the search kernels are launched on exact grids.
#include "common.hpp"

namespace apr {

namespace {

constexpr int kKeyBits = 30;  // 10 bits per axis

__device__ inline uint32_t spread10(uint32_t v)
{
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__device__ inline uint32_t quant10(double x, double lo, double L)
{
    double f = floor((x - lo) * (1024.0 / L));
    if (f < 0.0) f = 0.0;
    if (f > 1023.0) f = 1023.0;
    return (uint32_t)f;
}

__global__ void k_morton(const double *x, const double *y, const double *z, int64_t n, Box b,
                         uint32_t *keys, uint32_t *vals)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t qx = quant10(x[i], b.lo[0], b.L[0]);
    uint32_t qy = quant10(y[i], b.lo[1], b.L[1]);
    uint32_t qz = quant10(z[i], b.lo[2], b.L[2]);
    keys[i] = spread10(qx) | (spread10(qy) << 1) | (spread10(qz) << 2);
    vals[i] = (uint32_t)i;
}

constexpr int kLeafCap = 256;  // particles of an octree leaf before it is split

// Number of leading Morton levels (bit triplets) two 30-bit keys share, 0..10.
__device__ inline int common_levels(uint32_t a, uint32_t b)
{
    uint32_t x = a ^ b;
    return x == 0 ? 10 : (__clz(x) - 2) / 3;
}

__device__ inline int32_t wave_reduce_max(int32_t v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, kWave));
    return v;
}

__device__ inline int32_t wave_reduce_sum(int32_t v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Leaf starts.  i starts a leaf iff i = 0, or it starts a segment, or the
// cube shared by particles i-1 and i (level d = common_levels) holds more
// than kLeafCap particles: then the cube is split and i and i-1 fall into
// different children.  That cube holds more than C = kLeafCap particles iff
// some window of C + 1 consecutive particles around i-1, i lies inside it,
// i.e. iff g(j) = common_levels(key_j, key_{j+C}) >= d for some j in
// [i - C, i - 1] (the keys are sorted).  Equal keys never start a leaf (a
// leaf of more than C equal keys is cut into runs of 64 like any other).
//
// Tiles of kTile particles per workgroup of 1024 threads.  The window
// maximum comes from prefix and suffix maxima over aligned segments of C
// positions (a window of C spans at most two of them).
constexpr int kTileThreads = 1024;
constexpr int kTileItems = 4;
constexpr int kTile = kTileThreads * kTileItems;

__global__ __launch_bounds__(kTileThreads) void k_leaf_flags(const uint32_t *keys, int64_t n,
                                                             int seglev, uint32_t *flag,
                                                             int32_t *blast)
{
    constexpr int P = kTile + kLeafCap;  // position p <-> particle base - C + p
    constexpr int S = (P + kTileThreads - 1) / kTileThreads;
    __shared__ int8_t pre[P], suf[P];
    __shared__ int32_t red[kTileThreads / kWave];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int p = t; p < P; p += kTileThreads) {
        int64_t j = base - kLeafCap + p;
        int8_t g = (j >= 0 && j + kLeafCap < n)
                       ? (int8_t)common_levels(keys[j], keys[j + kLeafCap])
                       : (int8_t)-1;
        pre[p] = g;
        suf[p] = g;
    }
    __syncthreads();
    for (int o = 1; o < kLeafCap; o <<= 1) {
        int8_t a[S], b[S];
#pragma unroll
        for (int k = 0; k < S; ++k) {
            int p = t + k * kTileThreads;
            int r = p & (kLeafCap - 1);
            a[k] = (p < P && r >= o) ? pre[p - o] : (int8_t)-1;
            b[k] = (p < P && r + o < kLeafCap) ? suf[p + o] : (int8_t)-1;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < S; ++k) {
            int p = t + k * kTileThreads;
            if (p < P) {
                pre[p] = a[k] > pre[p] ? a[k] : pre[p];
                suf[p] = b[k] > suf[p] ? b[k] : suf[p];
            }
        }
        __syncthreads();
    }
    int32_t last = -1;
#pragma unroll
    for (int k = 0; k < kTileItems; ++k) {
        int q = t + k * kTileThreads;
        int64_t i = base + q;
        if (i >= n) continue;
        // window [i - C, i - 1] = positions [q, q + C - 1]
        int win = suf[q];
        if (q & (kLeafCap - 1)) win = max(win, (int)pre[q + kLeafCap - 1]);
        uint32_t f = 1;
        if (i > 0) {
            int d = common_levels(keys[i - 1], keys[i]);
            f = (d < seglev || (d < 10 && win >= d)) ? 1u : 0u;
        }
        flag[i] = f;
        if (f) last = (int32_t)i;
    }
    last = wave_reduce_max(last);
    if (lane_id() == 0) red[t / kWave] = last;
    __syncthreads();
    if (t == 0) {
        int32_t m = -1;
        for (int w = 0; w < kTileThreads / kWave; ++w) m = max(m, red[w]);
        blast[blockIdx.x] = m;
    }
}

// One workgroup: exclusive scan of v[0..nb) in place, with operator max
// (identity -1) or +; the total goes to *total when given, and with the
// build number `no` to the pinned host word *pin when given (one 64-bit
// store, so the host never reads a count with another build's number).
template <bool MAX>
__global__ __launch_bounds__(kTileThreads) void k_scan_blocks(int32_t *v, int64_t nb,
                                                              int32_t *total, uint64_t *pin,
                                                              uint32_t no)
{
    __shared__ int32_t red[kTileThreads / kWave + 1];
    const int t = threadIdx.x, lane = lane_id(), w = t / kWave;
    const int32_t id = MAX ? -1 : 0;
    auto op = [](int32_t a, int32_t b) { return MAX ? max(a, b) : a + b; };
    int64_t per = (nb + kTileThreads - 1) / kTileThreads;
    int64_t b0 = (int64_t)t * per, b1 = min(b0 + per, nb);
    int32_t s = id;
    for (int64_t k = b0; k < b1; ++k) s = op(s, v[k]);
    // exclusive scan of the thread sums
    int32_t incl = s;
    for (int o = 1; o < kWave; o <<= 1) {
        int32_t u = __shfl_up(incl, o, kWave);
        if (lane >= o) incl = op(incl, u);
    }
    if (lane == kWave - 1) red[w] = incl;
    __syncthreads();
    if (t == 0) {
        int32_t acc = id;
        for (int k = 0; k < kTileThreads / kWave; ++k) {
            int32_t x = red[k];
            red[k] = acc;
            acc = op(acc, x);
        }
        red[kTileThreads / kWave] = acc;
    }
    __syncthreads();
    int32_t ex = op(red[w], __shfl_up(incl, 1, kWave));
    if (lane == 0) ex = red[w];
    for (int64_t k = b0; k < b1; ++k) {
        int32_t x = v[k];
        v[k] = ex;
        ex = op(ex, x);
    }
    if (t == 0 && total) *total = red[kTileThreads / kWave];
    if (t == 0 && pin)
        __hip_atomic_store(pin, ((uint64_t)no << 32) | (uint32_t)red[kTileThreads / kWave],
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Cell starts inside leaves: every 64 particles from the leaf's first.  The
// leaf start of i is the largest leaf start <= i: an inclusive max-scan, the
// earlier tiles' part from carry[].  Writes cflag and the tile's cell count.
__global__ __launch_bounds__(kTileThreads) void k_cell_flags(const uint32_t *flag,
                                                             const int32_t *carry, int64_t n,
                                                             uint32_t *cflag, int32_t *bsum)
{
    __shared__ int32_t red[kTileThreads / kWave + 1];
    const int t = threadIdx.x, lane = lane_id(), w = t / kWave;
    const int64_t i0 = (int64_t)blockIdx.x * kTile + (int64_t)t * kTileItems;
    int32_t m[kTileItems];
    int32_t run = -1;
#pragma unroll
    for (int k = 0; k < kTileItems; ++k) {
        int64_t i = i0 + k;
        if (i < n && flag[i]) run = (int32_t)i;
        m[k] = run;
    }
    // exclusive max-scan of the threads' last starts
    int32_t incl = run;
    for (int o = 1; o < kWave; o <<= 1) {
        int32_t u = __shfl_up(incl, o, kWave);
        if (lane >= o) incl = max(incl, u);
    }
    if (lane == kWave - 1) red[w] = incl;
    __syncthreads();
    if (t == 0) {
        int32_t acc = carry[blockIdx.x];
        for (int k = 0; k < kTileThreads / kWave; ++k) {
            int32_t x = red[k];
            red[k] = acc;
            acc = max(acc, x);
        }
    }
    __syncthreads();
    int32_t prev = __shfl_up(incl, 1, kWave);
    int32_t before = lane > 0 ? max(red[w], prev) : red[w];
    int32_t cnt = 0;
#pragma unroll
    for (int k = 0; k < kTileItems; ++k) {
        int64_t i = i0 + k;
        if (i >= n) break;
        int32_t ls = max(before, m[k]);
        uint32_t cf = (i - ls) % kCell == 0 ? 1u : 0u;
        cflag[i] = cf;
        cnt += (int32_t)cf;
    }
    cnt = wave_reduce_sum(cnt);
    __syncthreads();
    if (lane == 0) red[w] = cnt;
    __syncthreads();
    if (t == 0) {
        int32_t s = 0;
        for (int k = 0; k < kTileThreads / kWave; ++k) s += red[k];
        bsum[blockIdx.x] = s;
    }
}

// Cell starts and the header (counts per tree level; nlev from the host).
__global__ __launch_bounds__(kTileThreads) void k_cell_start(const uint32_t *cflag,
                                                             const int32_t *boff, int64_t n,
                                                             int32_t *cell_start, Hdr *hdr,
                                                             int nlev)
{
    __shared__ int32_t red[kTileThreads / kWave + 1];
    const int t = threadIdx.x, lane = lane_id(), w = t / kWave;
    const int64_t i0 = (int64_t)blockIdx.x * kTile + (int64_t)t * kTileItems;
    uint32_t cf[kTileItems];
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < kTileItems; ++k) {
        int64_t i = i0 + k;
        cf[k] = i < n ? cflag[i] : 0u;
        s += (int32_t)cf[k];
    }
    int32_t incl = s;
    for (int o = 1; o < kWave; o <<= 1) {
        int32_t u = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += u;
    }
    if (lane == kWave - 1) red[w] = incl;
    __syncthreads();
    if (t == 0) {
        int32_t acc = boff[blockIdx.x];
        for (int k = 0; k < kTileThreads / kWave; ++k) {
            int32_t x = red[k];
            red[k] = acc;
            acc += x;
        }
    }
    __syncthreads();
    int32_t idx = red[w] + incl - s;
#pragma unroll
    for (int k = 0; k < kTileItems; ++k) {
        int64_t i = i0 + k;
        if (i >= n) break;
        if (cf[k]) cell_start[idx] = (int32_t)i;
        idx += (int32_t)cf[k];
        if (i == n - 1) {
            int64_t m = idx;
            cell_start[m] = (int32_t)n;
            hdr->ncells = (int32_t)m;
            hdr->nnode[0] = (int32_t)m;
            for (int l = 1; l <= kMaxLev; ++l) {
                m = l <= nlev ? (m + kFan - 1) / kFan : 0;
                hdr->nnode[l] = (int32_t)m;
            }
        }
    }
}

struct PermArgs {
    double *d[12];     // state double arrays (nullptr entries skipped)
    double *dt[12];    // temporaries
    int nd;
    int8_t *lev, *levt;
    int64_t *id, *idt;
    const uint32_t *perm;
    int64_t *perm_out;
    const float *fin;  // one float array gathered into another (no write-back)
    float *fout;
    int64_t n;
};

__global__ void k_gather(PermArgs a)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    uint32_t j = a.perm[i];
    for (int k = 0; k < a.nd; ++k) a.dt[k][i] = a.d[k][j];
    a.levt[i] = a.lev[j];
    a.idt[i] = a.id[j];
    if (a.perm_out) a.perm_out[i] = j;
    if (a.fin) a.fout[i] = a.fin[j];
}

__global__ void k_scatter_back(PermArgs a)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    for (int k = 0; k < a.nd; ++k) a.d[k][i] = a.dt[k][i];
    a.lev[i] = a.levt[i];
    a.id[i] = a.idt[i];
}

template <class T>
__device__ inline T wave_min(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, kWave));
    return v;
}
template <class T>
__device__ inline T wave_max(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

// Per-node kernels take one wavefront per item (4 per workgroup) and stride
// over the count the device holds, so any launch grid is correct.
#define APR_FOR_WAVE_ITEMS(j, count)                                                   \
    for (int64_t j = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave, \
                 j##_end = (count), j##_step = (int64_t)gridDim.x * (blockDim.x / kWave); \
         j < j##_end; j += j##_step)

// One wavefront per cell: bounding box, centre, rounded-up half extents and
// h_max; per particle the position relative to the cell centre and the
// normalised mass 2^-level, in the precision of the pair arithmetic.
template <class T>
__global__ __launch_bounds__(256) void k_cell_geo(const Hdr *hdr, const int32_t *cell_start,
                                                  const double *x, const double *y,
                                                  const double *z, const double *h,
                                                  const int8_t *level, Geo *cells,
                                                  vec4_t<T> *pm)
{
    const int lane = lane_id();
    APR_FOR_WAVE_ITEMS(c, hdr->ncells)
    {
        int32_t s0 = cell_start[c], s1 = cell_start[c + 1];
        int64_t i = s0 + lane;
        bool in = i < s1;
        double px = in ? x[i] : 0.0, py = in ? y[i] : 0.0, pz = in ? z[i] : 0.0;
        double ph = in ? h[i] : 0.0;
        double inf = __builtin_huge_val();
        double lx = wave_min(in ? px : inf), ly = wave_min(in ? py : inf),
               lz = wave_min(in ? pz : inf);
        double ux = wave_max(in ? px : -inf), uy = wave_max(in ? py : -inf),
               uz = wave_max(in ? pz : -inf);
        double hm = wave_max(ph);
        double cx = 0.5 * (lx + ux), cy = 0.5 * (ly + uy), cz = 0.5 * (lz + uz);
        if (lane == 0) {
            Geo g;
            g.cx = cx; g.cy = cy; g.cz = cz;
            g.ex = f_up(fmax(ux - cx, cx - lx));
            g.ey = f_up(fmax(uy - cy, cy - ly));
            g.ez = f_up(fmax(uz - cz, cz - lz));
            g.hmax = f_up(hm);
            cells[c] = g;
        }
        if (in) {
            vec4_t<T> v;
            v.x = (T)(px - cx);
            v.y = (T)(py - cy);
            v.z = (T)(pz - cz);
            v.w = (T)ldexp(1.0, -(int)level[i]);
            pm[i] = v;
        }
    }
}

// One wavefront per node: union of its (up to) 64 children.
__global__ __launch_bounds__(256) void k_tree_level(const Hdr *hdr, int lev, const Geo *child,
                                                    Geo *node)
{
    const int lane = lane_id();
    APR_FOR_WAVE_ITEMS(j, hdr->nnode[lev])
    {
        int64_t k = j * kFan + lane;
        bool in = k < hdr->nnode[lev - 1];
        double inf = __builtin_huge_val();
        Geo g;
        if (in) g = child[k];
        double lx = wave_min(in ? g.cx - (double)g.ex : inf);
        double ly = wave_min(in ? g.cy - (double)g.ey : inf);
        double lz = wave_min(in ? g.cz - (double)g.ez : inf);
        double ux = wave_max(in ? g.cx + (double)g.ex : -inf);
        double uy = wave_max(in ? g.cy + (double)g.ey : -inf);
        double uz = wave_max(in ? g.cz + (double)g.ez : -inf);
        float hm = wave_max(in ? g.hmax : 0.0f);
        if (lane == 0) {
            Geo o;
            o.cx = 0.5 * (lx + ux); o.cy = 0.5 * (ly + uy); o.cz = 0.5 * (lz + uz);
            o.ex = f_up(fmax(ux - o.cx, o.cx - lx));
            o.ey = f_up(fmax(uy - o.cy, o.cy - ly));
            o.ez = f_up(fmax(uz - o.cz, o.cz - lz));
            o.hmax = hm;
            node[j] = o;
        }
    }
}

// hmax of tree nodes only (boxes unchanged).
__global__ __launch_bounds__(256) void k_tree_hmax(const Hdr *hdr, int lev, const Geo *child,
                                                   Geo *node)
{
    const int lane = lane_id();
    APR_FOR_WAVE_ITEMS(j, hdr->nnode[lev])
    {
        int64_t k = j * kFan + lane;
        bool in = k < hdr->nnode[lev - 1];
        float hm = wave_max(in ? child[k].hmax : 0.0f);
        if (lane == 0) node[j].hmax = hm;
    }
}

// The cells' new hmax (one per cell, from the density pass) into their Geo and
// the level-1 nodes' hmax in the same pass: one wavefront per 64 cells (a
// level-1 node; node == nullptr when the tree has no level above the cells).
__global__ __launch_bounds__(256) void k_hmax_new_level1(const Hdr *hdr, const float *hmax_new,
                                                         Geo *cells, Geo *node)
{
    const int lane = lane_id();
    const int64_t nc = hdr->ncells;
    APR_FOR_WAVE_ITEMS(j, (nc + kFan - 1) / kFan)
    {
        int64_t k = j * kFan + lane;
        bool in = k < nc;
        float v = in ? hmax_new[k] : 0.0f;
        if (in) cells[k].hmax = v;
        float hm = wave_max(v);
        if (lane == 0 && node) node[j].hmax = hm;
    }
}

// Cells' hmax from a given h array.
__global__ __launch_bounds__(256) void k_cell_hmax(const Hdr *hdr, const int32_t *cell_start,
                                                   const double *h, Geo *cells)
{
    const int lane = lane_id();
    APR_FOR_WAVE_ITEMS(c, hdr->ncells)
    {
        int32_t s0 = cell_start[c], s1 = cell_start[c + 1];
        int64_t i = s0 + lane;
        double hm = wave_max(i < s1 ? h[i] : 0.0);
        if (lane == 0) cells[c].hmax = f_up(hm);
    }
}

}  // namespace

const Hdr *cell_hdr(apr_ctx *c) { return wsa<Hdr>(c, "cell_hdr", 1); }
const int32_t *cell_start(apr_ctx *c)
{
    return wsa<int32_t>(c, "cell_start", (size_t)c->node_cap[0] + 1);
}
Geo *cell_level(apr_ctx *c, int lev)
{
    static const char *names[kMaxLev + 1] = {"geo0", "geo1", "geo2", "geo3", "geo4", "geo5",
                                             "geo6"};
    return wsa<Geo>(c, names[lev], (size_t)c->node_cap[lev] + 1);
}

int refit_hmax_from_cells(apr_ctx *c)
{
    Hdr *hdr = wsa<Hdr>(c, "cell_hdr", 1);
    for (int k = 1; k <= c->nlev; ++k)
        hipLaunchKernelGGL(k_tree_hmax, dim3((unsigned)ceil_div(c->node_grid[k], 4)), dim3(256),
                           0, c->stream, hdr, k, cell_level(c, k - 1), cell_level(c, k));
    APR_LAUNCHED(c);
    return APR_OK;
}

int set_hmax_new(apr_ctx *c, const float *hmax_new)
{
    Hdr *hdr = wsa<Hdr>(c, "cell_hdr", 1);
    const int64_t g1 = ceil_div(c->node_grid[0], kFan);  // level-1 nodes (groups of 64 cells)
    hipLaunchKernelGGL(k_hmax_new_level1, dim3((unsigned)ceil_div(g1, 4)), dim3(256), 0,
                       c->stream, hdr, hmax_new, cell_level(c, 0),
                       c->nlev >= 1 ? cell_level(c, 1) : (Geo *)nullptr);
    for (int k = 2; k <= c->nlev; ++k)
        hipLaunchKernelGGL(k_tree_hmax, dim3((unsigned)ceil_div(c->node_grid[k], 4)), dim3(256),
                           0, c->stream, hdr, k, cell_level(c, k - 1), cell_level(c, k));
    APR_LAUNCHED(c);
    return APR_OK;
}

int cells_hmax_from(apr_ctx *c, const double *h, int64_t n)
{
    if (c->cells_n != n) return fail(c, APR_ERR_INVALID, "cells not built for this state");
    Hdr *hdr = wsa<Hdr>(c, "cell_hdr", 1);
    hipLaunchKernelGGL(k_cell_hmax, dim3((unsigned)ceil_div(c->node_grid[0], 4)), dim3(256), 0,
                       c->stream, hdr, cell_start(c), h, cell_level(c, 0));
    APR_LAUNCHED(c);
    return refit_hmax_from_cells(c);
}

static int build_cells_impl(apr_ctx *c, apr_state *s, int64_t *perm, bool keep_accel,
                            bool carry_divv);

int refit_cells(apr_ctx *c, apr_state *s)
{
    if (c->cells_n != s->n) return fail(c, APR_ERR_INVALID, "cells not built for this state");
    int tok = prof_begin(c, APR_PROF_CELLS);
    Hdr *hdr = wsa<Hdr>(c, "cell_hdr", 1);
    const int32_t *cs = cell_start(c);
    Geo *cells = cell_level(c, 0);
    const int64_t n = s->n;
    if (c->p.precision == APR_FP32) {
        float4 *pm = wsa<float4>(c, "pm32", (size_t)n);
        hipLaunchKernelGGL(k_cell_geo<float>, dim3((unsigned)ceil_div(c->node_grid[0], 4)),
                           dim3(256), 0, c->stream, hdr, cs, s->x, s->y, s->z, s->h, s->level,
                           cells, pm);
    } else {
        double4 *pm = wsa<double4>(c, "pm64", (size_t)n);
        hipLaunchKernelGGL(k_cell_geo<double>, dim3((unsigned)ceil_div(c->node_grid[0], 4)),
                           dim3(256), 0, c->stream, hdr, cs, s->x, s->y, s->z, s->h, s->level,
                           cells, pm);
    }
    for (int k = 1; k <= c->nlev; ++k)
        hipLaunchKernelGGL(k_tree_level, dim3((unsigned)ceil_div(c->node_grid[k], 4)), dim3(256),
                           0, c->stream, hdr, k, cell_level(c, k - 1), cell_level(c, k));
    APR_LAUNCHED(c);
    prof_end(c, tok);
    c->dens_n = -1;
    c->force_n = -1;
    return APR_OK;
}

int build_cells(apr_ctx *c, apr_state *s, int64_t *perm, bool keep_accel)
{
    if (!c->in_bins) c->bins_n = -1;  // a reorder the stored per-particle values miss
    // the last velocity divergence moves with the particles into "divv_prev"
    // (for the h predictor's extrapolation); "divv" is stale afterwards
    const bool dv = c->divv_n == s->n;
    c->divv_n = -1;
    c->divv_prev_n = -1;
    int tok = prof_begin(c, APR_PROF_CELLS);
    int rc = build_cells_impl(c, s, perm, keep_accel, dv);
    prof_end(c, tok);
    if (rc == APR_OK && dv) c->divv_prev_n = s->n;
    return rc;
}

static int build_cells_impl(apr_ctx *c, apr_state *s, int64_t *perm, bool keep_accel,
                            bool carry_divv)
{
    int64_t n = s->n;
    if (n <= 0) return fail(c, APR_ERR_INVALID, "empty state");
    if (n >= (int64_t)1 << 31) return fail(c, APR_ERR_INVALID, "too many particles");
    Box b = make_box(c->p);
    int seglev = c->p.periodic ? 2 : 3;
    // The cell count only sizes launch grids (the per-cell kernels take the
    // count on the device): use the newest count an earlier build has written
    // to the pinned word, scaled to n.
    {
        uint64_t v = __atomic_load_n(c->count_pin, __ATOMIC_ACQUIRE);
        uint32_t no = (uint32_t)(v >> 32);
        if (no != 0 && no > c->count_no && c->build_no - no < 16) {
            c->count_no = no;
            c->count_last = (int64_t)(uint32_t)v;
            c->count_last_n = c->build_n[no % 16];
        }
    }
    const uint32_t no = ++c->build_no;
    c->build_n[no % 16] = n;
    int64_t est = c->count_last > 0 && c->count_last_n > 0
                      ? std::max<int64_t>(1, c->count_last * n / c->count_last_n)
                      : 0;

    uint32_t *keys = wsa<uint32_t>(c, "mkeys", (size_t)n);
    uint32_t *vals = wsa<uint32_t>(c, "mvals", (size_t)n);
    uint32_t *lflag = wsa<uint32_t>(c, "leaf_flag", (size_t)n);
    uint32_t *cflag = wsa<uint32_t>(c, "cell_flag", (size_t)n);
    int32_t *blast = wsa<int32_t>(c, "tile_last", (size_t)ceil_div(n, kTile));
    int32_t *bsum = wsa<int32_t>(c, "tile_cells", (size_t)ceil_div(n, kTile));
    int32_t *tot = wsa<int32_t>(c, "cell_total", 2);
    Hdr *hdr = wsa<Hdr>(c, "cell_hdr", 1);
    if (!keys || !vals || !lflag || !cflag || !blast || !bsum || !tot || !hdr)
        return fail(c, APR_ERR_HIP, "cell workspace");
    unsigned g = (unsigned)ceil_div(n, 256);
    hipLaunchKernelGGL(k_morton, dim3(g), dim3(256), 0, c->stream, s->x, s->y, s->z, n, b, keys,
                       vals);
    APR_LAUNCHED(c);
    int rc = radix_sort_u32(c, keys, vals, n, kKeyBits, &keys, &vals);
    if (rc) return rc;

    // permute the state in place through temporaries
    PermArgs pa;
    std::memset(&pa, 0, sizeof(pa));
    double *arrs[12] = {s->x, s->y, s->z, s->vx, s->vy, s->vz, s->u, s->h,
                        keep_accel ? s->ax : nullptr, keep_accel ? s->ay : nullptr,
                        keep_accel ? s->az : nullptr, keep_accel ? s->dudt : nullptr};
    static const char *tn[12] = {"pt0", "pt1", "pt2", "pt3", "pt4", "pt5",
                                 "pt6", "pt7", "pt8", "pt9", "pt10", "pt11"};
    for (int k = 0; k < 12; ++k) {
        if (!arrs[k]) continue;
        pa.d[pa.nd] = arrs[k];
        pa.dt[pa.nd] = wsa<double>(c, tn[pa.nd], (size_t)n);
        if (!pa.dt[pa.nd]) return fail(c, APR_ERR_HIP, "permute workspace");
        pa.nd += 1;
    }
    pa.lev = s->level;
    pa.levt = wsa<int8_t>(c, "pt_lev", (size_t)n);
    pa.id = s->id;
    pa.idt = wsa<int64_t>(c, "pt_id", (size_t)n);
    pa.perm = vals;
    pa.perm_out = perm;
    pa.n = n;
    if (carry_divv) {
        pa.fin = wsa<float>(c, "divv", (size_t)n);
        pa.fout = wsa<float>(c, "divv_prev", (size_t)n);
        if (!pa.fin || !pa.fout) return fail(c, APR_ERR_HIP, "permute workspace");
    }
    hipLaunchKernelGGL(k_gather, dim3(g), dim3(256), 0, c->stream, pa);
    hipLaunchKernelGGL(k_scatter_back, dim3(g), dim3(256), 0, c->stream, pa);
    APR_LAUNCHED(c);

    // octree leaves, then cells of <= 64 within each leaf
    int64_t nt = ceil_div(n, kTile);
    unsigned gt = (unsigned)nt;
    hipLaunchKernelGGL(k_leaf_flags, dim3(gt), dim3(kTileThreads), 0, c->stream, keys, n, seglev,
                       lflag, blast);
    hipLaunchKernelGGL(k_scan_blocks<true>, dim3(1), dim3(kTileThreads), 0, c->stream, blast, nt,
                       (int32_t *)nullptr, (uint64_t *)nullptr, 0u);
    hipLaunchKernelGGL(k_cell_flags, dim3(gt), dim3(kTileThreads), 0, c->stream, lflag, blast, n,
                       cflag, bsum);
    hipLaunchKernelGGL(k_scan_blocks<false>, dim3(1), dim3(kTileThreads), 0, c->stream, bsum, nt,
                       tot, c->count_pin, no);
    APR_LAUNCHED(c);
    // the first build of a context waits for its count
    if (est <= 0) {
        APR_HIP(c, hipStreamSynchronize(c->stream));
        uint64_t v = __atomic_load_n(c->count_pin, __ATOMIC_ACQUIRE);
        est = (int64_t)(uint32_t)v;
        if ((uint32_t)(v >> 32) != no || est < 1 || est > n)
            return fail(c, APR_ERR_HIP, "cell count out of range");
        c->count_no = no;
        c->count_last = est;
        c->count_last_n = n;
    }
    // buffers: at most one cell per particle; grids: the estimate with a margin.
    // Levels: enough for n cells, so the top level never has more than kFan
    // nodes (with fewer cells the upper levels hold a single node).
    int64_t grid = c->grid_set > 0 ? c->grid_set : std::min<int64_t>(n, est + est / 8 + 64);
    int nlev = 0;
    int64_t m = n;
    c->node_cap[0] = n;
    c->node_grid[0] = grid;
    while (m > kFan) {
        m = ceil_div(m, kFan);
        grid = ceil_div(grid, kFan);
        nlev += 1;
        c->node_cap[nlev] = m;
        c->node_grid[nlev] = grid;
    }
    if (nlev > kMaxLev) return fail(c, APR_ERR_INVALID, "too many particles for the tree");
    c->nlev = nlev;
    int32_t *cs = wsa<int32_t>(c, "cell_start", (size_t)c->node_cap[0] + 1);
    if (!cs) return fail(c, APR_ERR_HIP, "cell workspace");
    hipLaunchKernelGGL(k_cell_start, dim3(gt), dim3(kTileThreads), 0, c->stream, cflag, bsum, n,
                       cs, hdr, nlev);
    APR_LAUNCHED(c);

    Geo *cells = cell_level(c, 0);
    if (c->p.precision == APR_FP32) {
        float4 *pm = wsa<float4>(c, "pm32", (size_t)n);
        hipLaunchKernelGGL(k_cell_geo<float>, dim3((unsigned)ceil_div(c->node_grid[0], 4)),
                           dim3(256), 0, c->stream, hdr, cs, s->x, s->y, s->z, s->h, s->level,
                           cells, pm);
    } else {
        double4 *pm = wsa<double4>(c, "pm64", (size_t)n);
        hipLaunchKernelGGL(k_cell_geo<double>, dim3((unsigned)ceil_div(c->node_grid[0], 4)),
                           dim3(256), 0, c->stream, hdr, cs, s->x, s->y, s->z, s->h, s->level,
                           cells, pm);
    }
    APR_LAUNCHED(c);
    for (int k = 1; k <= nlev; ++k)
        hipLaunchKernelGGL(k_tree_level, dim3((unsigned)ceil_div(c->node_grid[k], 4)), dim3(256),
                           0, c->stream, hdr, k, cell_level(c, k - 1), cell_level(c, k));
    APR_LAUNCHED(c);
    c->cells_n = n;
    c->dens_n = -1;
    c->force_n = -1;
    return APR_OK;
}

}  // namespace apr
