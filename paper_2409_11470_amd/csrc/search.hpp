// Device-side neighbour-candidate search shared by the density, force and
// adjoint kernels.
//
// Work unit: one workgroup of 4 wavefronts per target cell (<= 64 particles).
//  1. traverse: wavefront 0 walks the 64-ary cell tree breadth-first; at each
//     level one wavefront instruction tests the 64 children of a frontier
//     node, and ballot + popcount append the hits in order (deterministic).
//  2. stage: the candidate cells' particles that can interact with the target
//     cell are copied to LDS, with positions moved into the target cell's
//     frame (FP64 cell-centre difference, minimum image, rounded once to the
//     pair precision).  Counted per candidate cell first, then written at the
//     prefix offsets, so the staged order is the candidate order (fixed).
//  3. sub-block lists: the 64 targets form 16 sub-blocks of 4; a wavefront
//     serves one sub-block at a time with 16 lanes per target, and the staged
//     candidates that can reach the sub-block are listed (u16 LDS indices).
//  If the staged set or a sub-block list does not fit in LDS, that work reads
//  the candidate cells straight from global memory instead (same arithmetic,
//  slower), so no capacity limit changes a result.
#pragma once

#include "common.hpp"

namespace apr {

constexpr int kSearchThreads = 256;
constexpr int kWaves = kSearchThreads / kWave;
constexpr int kCandCap = 1024;   // candidate cells per target cell
constexpr int kSubCap = 512;     // staged candidates per sub-block
constexpr int kGroup = 16;       // lanes per target

struct Tree {
    const Hdr *hdr;
    const int32_t *cs;           // cell starts [ncells + 1]
    const Geo *lev[kMaxLev + 1]; // lev[0] = cells
    int nlev;
    Box box;
};

// Orders LDS traffic between the lanes of one wavefront (a compiler and
// memory fence at wavefront scope; the wavefront runs in lockstep).
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Breadth-first traversal by one wavefront.  Keeps the nodes whose box lies
// within R of the target box (or, with sym, within max(R, 2 hmax_node)).
// Returns the number of candidate cells written to A (<= kCandCap; sets
// *overflow if more were found).
__device__ inline int traverse(const Tree &t, const Geo &tg, double R, bool sym, int32_t *A,
                               int32_t *B, int *overflow)
{
    int lane = lane_id();
    int top = t.nlev;
    int ntop = t.hdr->nnode[top];
    double R2 = R * R;
    int nf = 0;
    // the top level (<= 64 nodes) is tested directly
    {
        bool in = lane < ntop;
        bool hit = false;
        if (in) {
            Geo g = t.lev[top][lane];
            double r = sym ? fmax(R, 2.0 * (double)g.hmax) : R;
            hit = gap2(tg, g, t.box) < (sym ? r * r : R2);
        }
        uint64_t m = __ballot(hit);
        if (hit) A[__popcll(m & lanemask_lt())] = lane;
        nf = __popcll(m);
        wave_sync();
    }
    int32_t *cur = A, *nxt = B;
    for (int lev = top; lev >= 1; --lev) {
        int nchild = t.hdr->nnode[lev - 1];
        const Geo *cg = t.lev[lev - 1];
        int nn = 0;
        for (int f = 0; f < nf; ++f) {
            int64_t ch = (int64_t)cur[f] * kFan + lane;
            bool hit = false;
            if (ch < nchild) {
                Geo g = cg[ch];
                double r = sym ? fmax(R, 2.0 * (double)g.hmax) : R;
                hit = gap2(tg, g, t.box) < r * r;
            }
            uint64_t m = __ballot(hit);
            int pos = nn + __popcll(m & lanemask_lt());
            if (hit && pos < kCandCap) nxt[pos] = (int32_t)ch;
            nn += __popcll(m);
        }
        if (nn > kCandCap) {
            *overflow = 1;
            nn = kCandCap;
        }
        wave_sync();
        int32_t *tmp = cur;
        cur = nxt;
        nxt = tmp;
        nf = nn;
    }
    // make sure the result sits in A
    if (cur != A) {
        for (int i = lane; i < nf; i += kWave) A[i] = cur[i];
        wave_sync();
    }
    return nf;
}

// In-place exclusive prefix sum of cnt[0..n) by one wavefront; returns the total.
__device__ inline int wave_excl_scan_lds(int32_t *cnt, int n)
{
    int lane = lane_id();
    int carry = 0;
    for (int base = 0; base < n; base += kWave) {
        int i = base + lane;
        int v = i < n ? cnt[i] : 0;
        int incl = v;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            int t = __shfl_up(incl, o, kWave);
            if (lane >= o) incl += t;
        }
        if (i < n) cnt[i] = carry + incl - v;
        carry += __shfl(incl, kWave - 1, kWave);
    }
    wave_sync();
    return carry;
}

// Centre difference (candidate cell - target cell), minimum image, in FP64.
__device__ inline void cell_shift(const Geo &cand, const Geo &tg, const Box &b, double *s)
{
    s[0] = min_image(cand.cx - tg.cx, b.L[0], b.periodic);
    s[1] = min_image(cand.cy - tg.cy, b.L[1], b.periodic);
    s[2] = min_image(cand.cz - tg.cz, b.L[2], b.periodic);
}

// Squared distance from a point to an axis-aligned box (centre c, half e).
template <class T>
__device__ inline T pt_box_d2(T x, T y, T z, T cx, T cy, T cz, T ex, T ey, T ez)
{
    T gx = fabs(x - cx) - ex, gy = fabs(y - cy) - ey, gz = fabs(z - cz) - ez;
    gx = gx > T(0) ? gx : T(0);
    gy = gy > T(0) ? gy : T(0);
    gz = gz > T(0) ? gz : T(0);
    return gx * gx + gy * gy + gz * gz;
}

template <class T>
__device__ inline T wmax16(T v)
{
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) {
        T u = __shfl_xor(v, o, kGroup);
        v = v > u ? v : u;
    }
    return v;
}
template <class T>
__device__ inline T wmin16(T v)
{
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) {
        T u = __shfl_xor(v, o, kGroup);
        v = v < u ? v : u;
    }
    return v;
}
template <class T>
__device__ inline T wsum16(T v)
{
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o, kGroup);
    return v;
}

// Max over the 4 groups of a wavefront (lanes 0, 16, 32, 48 hold group values).
template <class T>
__device__ inline T wmax_groups(T v)
{
    T u = __shfl_xor(v, 16, kWave);
    v = v > u ? v : u;
    u = __shfl_xor(v, 32, kWave);
    return v > u ? v : u;
}
template <class T>
__device__ inline T wmin_groups(T v)
{
    T u = __shfl_xor(v, 16, kWave);
    v = v < u ? v : u;
    u = __shfl_xor(v, 32, kWave);
    return v < u ? v : u;
}

// Compensated (Kahan) accumulation in the pair precision: the sum is s - c.
template <class T>
struct Acc {
    T s, c;
    __device__ void zero()
    {
        s = T(0);
        c = T(0);
    }
    __device__ void add(T x)
    {
        T y = x - c;
        T t = s + y;
        c = (t - s) - y;
        s = t;
    }
    // combine with the 15 other lanes of the group (TwoSum on the partials)
    __device__ void reduce16()
    {
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) {
            T s2 = __shfl_xor(s, o, kGroup), c2 = __shfl_xor(c, o, kGroup);
            T t = s + s2;
            T bb = t - s;
            T err = (s - (t - bb)) + (s2 - bb);
            c = c + c2 - err;
            s = t;
        }
    }
    __device__ double value() const { return (double)s - (double)c; }
};

}  // namespace apr
