// Device-side neighbour-candidate search shared by the density, force and
// adjoint kernels.
//
// Work unit: one workgroup of 4 wavefronts per target cell (<= 64 particles).
//  1. walk: wavefront 0 walks the 64-ary cell tree depth-first; one wavefront
//     instruction tests the 64 children of a node, and ballot + popcount
//     append the hit cells in order (deterministic).  The walk pauses when the
//     candidate buffer is full, the candidates so far are processed, and it
//     resumes: the number of candidate cells is unbounded.
//  2. stage: the candidate cells' particles that can interact with the target
//     cell are copied to LDS, with positions moved into the target cell's
//     frame (FP64 absolute position minus the target cell's centre, minimum
//     image of the cell pair, rounded once to the pair precision).  Counted
//     per candidate cell first, then written at the prefix offsets, so the
//     staged order is the candidate order (fixed).
//  3. sub-block lists: the 64 targets form 16 sub-blocks of 4; a wavefront
//     serves one sub-block at a time with 16 lanes per target, and the staged
//     candidates that can reach the sub-block are listed (u16 LDS indices).
//  4. per-target lists: each target's 16 lanes keep, from its sub-block list,
//     the candidates inside its own support (with margin); the pair loops walk
//     only those.
//  If the staged set or a sub-block list does not fit in LDS, that work reads
//  the candidate cells straight from global memory instead (same arithmetic,
//  slower), so no capacity limit changes a result.
#pragma once

#include "common.hpp"

namespace apr {

constexpr int kSearchThreads = 256;
constexpr int kWaves = kSearchThreads / kWave;
constexpr int kRestGrid = 256;   // workgroups of a search kernel's REST launch
constexpr int kCandCap = 256;    // candidate cells per chunk of the walk
constexpr int kSubCap = 512;     // staged candidates per sub-block
constexpr int kListLanes = 16;   // lanes per target while building the per-target lists
constexpr int kLanes = 4;        // lanes per target (one target per lane group of 4)
constexpr int kTCap = 128;       // per-target candidate list (u16 LDS indices)
// Workgroups per CU the density and force kernels are compiled for: the FP32
// kernels fit 4 (LDS <= 40 KB, <= 128 VGPRs) to hide the latency of the
// candidate loads and LDS walks; the FP64 ones fit 3 (<= 168 VGPRs, a few
// spills), which hides more latency than 2 without spills does.
template <class T>
constexpr int kBlocksPerCU = sizeof(T) == 4 ? 4 : 3;

// Orders LDS traffic between the lanes of one wavefront (a compiler and
// memory fence at wavefront scope; the wavefront runs in lockstep).
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct Tree {
    const Hdr *hdr;
    const int32_t *cs;           // cell starts [ncells + 1]
    const Geo *lev[kMaxLev + 1]; // lev[0] = cells
    int nlev;
    Box box;
    // the state the cells were built on (cell order): FP64 positions for the
    // staged coordinates and, with ph, the exact support test near its edge
    const double *px, *py, *pz, *ph;
};

// ------------------------------------------------------------ exact support
// Membership in a support is decided like the FP64 neighbour export: the
// minimum-image separation of the absolute positions, r^2 = dx*dx + dy*dy +
// dz*dz summed left to right with every product and sum rounded on its own
// (no contraction), tested strictly against (2 h)^2.  The pair loops test in
// the pair precision on cell-frame coordinates and take this FP64 decision
// only inside a guard band about the edge, where the rounding of the
// pair-precision test could decide otherwise.
__device__ inline double sep_exact(double a, double b, double L, int periodic)
{
#pragma clang fp contract(off)
    double d = a - b;
    if (periodic) {
        if (d > 0.5 * L) d -= L;
        else if (d < -0.5 * L) d += L;
    }
    return d;
}

__device__ inline double r2_exact(const Tree &t, int64_t a, int64_t b)
{
#pragma clang fp contract(off)
    double dx = sep_exact(t.px[a], t.px[b], t.box.L[0], t.box.periodic);
    double dy = sep_exact(t.py[a], t.py[b], t.box.L[1], t.box.periodic);
    double dz = sep_exact(t.pz[a], t.pz[b], t.box.L[2], t.box.periodic);
    return dx * dx + dy * dy + dz * dz;
}

// r_ab^2 < (2 h)^2, h in FP64, evaluated exactly as above.
__device__ inline bool inside_exact(double r2, double h)
{
#pragma clang fp contract(off)
    double R = 2.0 * h;
    return r2 < R * R;
}

// Guard band of the pair-precision support test, in units of r^2: for a
// target at cell-frame position t (|t|_1 = mt) and support radius R,
//   band = kBand * R * (mt + 2 R).
// The staged coordinates are rounded once from FP64 (relative error 2^-24 in
// FP32), so a separation near R carries an error below about
// 2^-23 (|t|_inf + R) per component and r^2 one below about
// 2^-21 R (mt + R); kBand leaves a factor of 8 over that.  The FP64 form
// rounds the same way at 2^-53 (and at most 2^-53 L more in a periodic
// image), covered by its kBand with the same margin.
template <class T>
constexpr T kBand = sizeof(T) == 4 ? T(1.0 / (1 << 18)) : T(1.0 / (1ll << 44));

template <class T>
__device__ inline T edge_band(const vec4_t<T> &t, T R)
{
    return kBand<T> * R * (fabs(t.x) + fabs(t.y) + fabs(t.z) + T(2) * R);
}

// The slot of a staged candidate rides in a component the pair sums never
// read (bit pattern of an int32 or int64).
__device__ inline float slot_bits(float, int64_t i) { return __int_as_float((int32_t)i); }
__device__ inline double slot_bits(double, int64_t i) { return __longlong_as_double(i); }
__device__ inline int64_t slot_of(float v) { return (int64_t)__float_as_int(v); }
__device__ inline int64_t slot_of(double v) { return (int64_t)__double_as_longlong(v); }

// Resumable depth-first walk of the cell tree by one wavefront, handing out
// the candidate cells in chunks (in Morton order, the order of the cells), so
// that no candidate capacity limits a search.  A node is kept if its box lies
// within R of the target box (or, with sym, within max(R, 2 hmax_node)).
// State per level: the hit mask of the 64 children of the node being
// expanded there and the id of child 0.  Lives in LDS; wavefront-uniform.
struct Walk {
    uint64_t mask[kMaxLev + 1];
    int32_t base[kMaxLev + 1];
    int depth;  // level of the deepest pending mask; > nlev when finished
};

__device__ inline bool node_hit(const Geo &g, const Geo &tg, const Box &box, double R, bool sym)
{
    double r = sym ? fmax(R, 2.0 * (double)g.hmax) : R;
    return gap2(tg, g, box) < r * r;
}

// Starts the walk: tests the top-level nodes (<= 64).
__device__ inline void walk_init(const Tree &t, const Geo &tg, double R, bool sym, Walk *W)
{
    int lane = lane_id(), top = t.nlev;
    bool hit = lane < t.hdr->nnode[top] && node_hit(t.lev[top][lane], tg, t.box, R, sym);
    uint64_t m = __ballot(hit);
    wave_sync();
    if (lane == 0) {
        W->mask[top] = m;
        W->base[top] = 0;
        W->depth = top;
    }
    wave_sync();
}

__device__ inline bool walk_done(const Tree &t, const Walk *W) { return W->depth > t.nlev; }

// Appends the next candidate cells to A (room for cap >= 64), whole groups of
// siblings at a time, and returns their number; 0 once the walk is finished.
__device__ inline int walk_next(const Tree &t, const Geo &tg, double R, bool sym, Walk *W,
                                int32_t *A, int cap)
{
    int lane = lane_id();
    int n = 0;
    int d = W->depth;
    while (d <= t.nlev) {
        uint64_t m = W->mask[d];
        if (m == 0) {
            d += 1;
            continue;
        }
        if (d == 0) {
            int k = __popcll(m);
            if (n + k > cap) break;  // the caller takes this chunk first
            if ((m >> lane) & 1ull) A[n + __popcll(m & lanemask_lt())] = W->base[0] + lane;
            n += k;
            wave_sync();
            if (lane == 0) W->mask[0] = 0;
            wave_sync();
            d = 1;
            continue;
        }
        // expand the first pending node of level d
        int slot = __ffsll((unsigned long long)m) - 1;
        int32_t node = W->base[d] + slot;
        int64_t ch = (int64_t)node * kFan + lane;
        bool hit = ch < t.hdr->nnode[d - 1] && node_hit(t.lev[d - 1][ch], tg, t.box, R, sym);
        uint64_t cm = __ballot(hit);
        wave_sync();
        if (lane == 0) {
            W->mask[d] = m & (m - 1);
            W->mask[d - 1] = cm;
            W->base[d - 1] = node * kFan;
        }
        wave_sync();
        d -= 1;
    }
    wave_sync();
    if (lane == 0) W->depth = d;
    wave_sync();
    return n;
}

// Candidate cells of every cell from a walk ahead of the search kernel (see
// candidates.hip): cand[cell * kCandCap + k], k < ncand[cell]; ncand -1 means
// "walk yourself", and so do cells >= cap (the lists are sized from the host's
// estimate of the cell count).  The walk used radius rfac * hmax of the cell.
struct CandList {
    const int32_t *cand = nullptr;
    const int32_t *ncand = nullptr;
    double rfac = 0.0;
    int64_t cap = 0;
};
int cand_pre(apr_ctx *c, const Tree &tr, bool sym, double rfac, CandList *out,
             const uint8_t *active = nullptr);

// In-place exclusive prefix sum of cnt[0..n) by one wavefront; returns the total.
__device__ inline int wave_excl_scan_lds(int32_t *cnt, int n)
{
    int lane = lane_id();
    int carry = 0;
    for (int base = 0; base < n; base += kWave) {
        int i = base + lane;
        int v = i < n ? cnt[i] : 0;
        // inclusive scan by DPP: within each 16-lane row by shifts of 1, 2,
        // 4, 8 (lanes with no source add 0), then row 0's total into row 1
        // and row 2's into row 3, then lane 31's prefix into rows 2 and 3
        int incl = v;
        incl += __builtin_amdgcn_update_dpp(0, incl, 0x111, 0xF, 0xF, false);  // row_shr:1
        incl += __builtin_amdgcn_update_dpp(0, incl, 0x112, 0xF, 0xF, false);  // row_shr:2
        incl += __builtin_amdgcn_update_dpp(0, incl, 0x114, 0xF, 0xF, false);  // row_shr:4
        incl += __builtin_amdgcn_update_dpp(0, incl, 0x118, 0xF, 0xF, false);  // row_shr:8
        incl += __builtin_amdgcn_update_dpp(0, incl, 0x142, 0xA, 0xF, false);  // row_bcast:15
        incl += __builtin_amdgcn_update_dpp(0, incl, 0x143, 0xC, 0xF, false);  // row_bcast:31
        if (i < n) cnt[i] = carry + incl - v;
        carry += __builtin_amdgcn_readlane(incl, kWave - 1);
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

// Reductions over the 4 lanes of a target.
template <class T>
__device__ inline T sum4(T v)
{
    v += lane_xor<1>(v);
    v += lane_xor<2>(v);
    return v;
}
template <class T>
__device__ inline T min4(T v)
{
    T u = lane_xor<1>(v);
    v = v < u ? v : u;
    u = lane_xor<2>(v);
    return v < u ? v : u;
}
template <class T>
__device__ inline T max4(T v)
{
    T u = lane_xor<1>(v);
    v = v > u ? v : u;
    u = lane_xor<2>(v);
    return v > u ? v : u;
}
// Max / min over the whole wavefront.
// One butterfly step of a max / min over lanes O apart: within rows the
// partner's value (op(own, partner)), across rows and halves the ordered
// pair (so partner lanes agree bitwise).
template <int O, bool MAX, class T>
__device__ inline T minmax_step(T v)
{
    auto op = [](T x, T y) { return MAX ? (x > y ? x : y) : (x < y ? x : y); };
    if constexpr (O >= 16) {
        T lo, hi;
        lane_pair<O>(v, lo, hi);
        return op(lo, hi);
    } else {
        return op(v, lane_xor<O>(v));
    }
}
// Max / min over the lanes j, j + G, j + 2G, ... of the wavefront (G = 1: over
// all of it), which every lane ends with.
template <int G, bool MAX, class T>
__device__ inline T wminmax_lanes(T v)
{
    if constexpr (G <= 1) v = minmax_step<1, MAX>(v);
    if constexpr (G <= 2) v = minmax_step<2, MAX>(v);
    if constexpr (G <= 4) v = minmax_step<4, MAX>(v);
    if constexpr (G <= 8) v = minmax_step<8, MAX>(v);
    if constexpr (G <= 16) v = minmax_step<16, MAX>(v);
    return minmax_step<32, MAX>(v);
}
template <int G, class T>
__device__ inline T wmax_lanes(T v)
{
    return wminmax_lanes<G, true>(v);
}
template <int G, class T>
__device__ inline T wmin_lanes(T v)
{
    return wminmax_lanes<G, false>(v);
}
template <class T>
__device__ inline T wave_max64(T v)
{
    return wmax_lanes<1>(v);
}
template <class T>
__device__ inline T wave_min64(T v)
{
    return wmin_lanes<1>(v);
}

// The targets of each wavefront (16 of a cell's 64) as a box [lo, hi] in the
// cell frame with its own reach R: a candidate is staged only if it lies
// within reach of some wavefront's box.  For cells of mixed h this is much
// tighter than one radius (from the largest h) around the whole cell.
template <class T>
struct WaveBoxes {
    T lo[kWaves][3], hi[kWaves][3];
    T R2[kWaves];   // < 0: the wavefront has no target
};

// Every thread calls it; (x, y, z) is this lane's target position, valid if
// the lane has a target.  Writes the wavefront's box (not R2) to B.
template <class T>
__device__ inline void wave_box(WaveBoxes<T> *B, bool valid, T x, T y, T z)
{
    const T big = T(3.0e38);
    T lx = wave_min64(valid ? x : big), ly = wave_min64(valid ? y : big),
      lz = wave_min64(valid ? z : big);
    T hx = wave_max64(valid ? x : -big), hy = wave_max64(valid ? y : -big),
      hz = wave_max64(valid ? z : -big);
    if (lane_id() == 0) {
        int w = wave_id();
        B->lo[w][0] = lx; B->lo[w][1] = ly; B->lo[w][2] = lz;
        B->hi[w][0] = hx; B->hi[w][1] = hy; B->hi[w][2] = hz;
    }
}

// Squared distance of a point to the box [lo, hi].
template <class T>
__device__ inline T pt_lohi_d2(T x, T y, T z, const T *lo, const T *hi)
{
    T gx = fmax(fmax(lo[0] - x, x - hi[0]), T(0));
    T gy = fmax(fmax(lo[1] - y, y - hi[1]), T(0));
    T gz = fmax(fmax(lo[2] - z, z - hi[2]), T(0));
    return gx * gx + gy * gy + gz * gz;
}

// Within reach of some wavefront's targets: d2_w < R2_w or, with SYM, within
// the candidate's own support, d2_w / h_b^2 < 4 (hb2 = 1/h_b^2).
// The wavefront loop is kept rolled so that the boxes are read from LDS at
// each test (broadcast reads) instead of living in registers across the
// staging loops (28 values).
template <class T, bool SYM>
__device__ inline bool wave_reach(const WaveBoxes<T> &B, T x, T y, T z, T hb2)
{
    bool hit = false;
#pragma unroll 1
    for (int k = 0; k < kWaves; ++k) {
        T r2 = B.R2[k];
        T d2 = pt_lohi_d2<T>(x, y, z, B.lo[k], B.hi[k]);
        // bitwise, no branches: most candidates are tested against every box anyway
        hit = hit | ((r2 >= T(0)) & ((d2 < r2) | (SYM & (d2 * hb2 < T(4)))));
    }
    return hit;
}

// What staging needs of one candidate cell: its first particle, its size
// (at most kCell) and the offset from its frame to the target cell's frame
// (minimum image), read once for all candidates of a chunk so that the
// counting and staging loops wait on one global load per cell, not three
// chained ones.
template <class T>
struct CandMeta {
    T sx, sy, sz;
    int32_t b0;
    uint32_t wrap;  // periodic image of the candidate cell, 2 bits per axis:
                    // 1 adds the box length, 2 subtracts it
};
template <class T>
struct MetaBuf {
    CandMeta<T> m[kCandCap];
    uint8_t bn[kCandCap];
};
// The per-target lists and the candidates' metadata are never live at once
// (metadata: from the walk to the end of staging; lists: from their build to
// the next staging), so they share LDS.
template <class T, int CAP>
union ListsMeta {
    uint16_t tls[kCell][CAP];
    MetaBuf<T> meta;
};

// All threads of the workgroup fill mb for candidates [0, nc) of sA; the
// caller synchronises before reading it.
template <class T>
__device__ inline void load_meta(const Tree &tr, const Geo &tg, const int32_t *sA, int nc,
                                 MetaBuf<T> *mb)
{
    for (int ci = threadIdx.x; ci < nc; ci += kSearchThreads) {
        int cc = sA[ci];
        int32_t b0 = tr.cs[cc], b1 = tr.cs[cc + 1];
        const Geo g = tr.lev[0][cc];
        double sh[3];
        cell_shift(g, tg, tr.box, sh);
        const double raw[3] = {g.cx - tg.cx, g.cy - tg.cy, g.cz - tg.cz};
        CandMeta<T> x;
        x.sx = (T)sh[0];
        x.sy = (T)sh[1];
        x.sz = (T)sh[2];
        x.b0 = b0;
        x.wrap = 0;
        for (int k = 0; k < 3; ++k)
            x.wrap |= (sh[k] > raw[k] ? 1u : (sh[k] < raw[k] ? 2u : 0u)) << (2 * k);
        mb->m[ci] = x;
        mb->bn[ci] = (uint8_t)(b1 - b0);
    }
}

// Position of candidate particle b in the target cell's frame (centre tg),
// rounded once from FP64: (x_b + image shift) - c.
template <class T>
__device__ inline void stage_pos(const Tree &tr, const Geo &tg, uint32_t wrap, int64_t b,
                                 vec4_t<T> &p)
{
#pragma clang fp contract(off)
    const Box &bx = tr.box;
    // the image shift is selected first and then added, so that a wrap
    // common to the wavefront (a scalar) costs a select, not a branch that
    // would wait for each coordinate's load in turn
    auto img = [&](double v, int k) {
        const uint32_t c = (wrap >> (2 * k)) & 3u;
        const double sh = c == 1u ? bx.L[k] : (c == 2u ? -bx.L[k] : 0.0);
        return v + sh;
    };
    p.x = (T)(img(tr.px[b], 0) - tg.cx);
    p.y = (T)(img(tr.py[b], 1) - tg.cy);
    p.z = (T)(img(tr.pz[b], 2) - tg.cz);
}

// One staged entry as a single vector read: the pair loops test the
// position before they use the mass, and a per-field read lets the compiler
// defer the mass into the taken branch, one more LDS round trip per pair.
template <class T>
__device__ inline vec4_t<T> lds_ld4(const vec4_t<T> *p)
{
    typedef T n4 __attribute__((ext_vector_type(4)));
    const n4 v = *reinterpret_cast<const n4 *>(p);
    vec4_t<T> r;
    r.x = v.x;
    r.y = v.y;
    r.z = v.z;
    r.w = v.w;
    return r;
}

// Staging and the per-block box tests keep a relative slack over the exact
// criteria: a candidate that the exact per-target test accepts must pass them
// whatever the rounding of the (differently grouped) distance sums.
// The slack also covers the guard band of the support test (kBand) for
// targets within 126 R of their cell's centre (|t|_1 < 126 R); the density
// kernel counts targets beyond that (ST_BAND).
template <class T>
constexpr T kReachSlack = T(1) + T(1.0 / (1 << 10));

// Square root and reciprocal square root in the pair precision: the FP32
// form uses the hardware v_sqrt_f32 / v_rsq_f32 (about 1 ulp), the FP64 form
// the correctly rounded library functions.
__device__ inline float psqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ inline double psqrt(double x) { return sqrt(x); }
__device__ inline float prsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline double prsqrt(double x) { return 1.0 / sqrt(x); }

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
    // combine with the other lanes of a width-W group (TwoSum on the partials)
    template <int W>
    __device__ void reduce()
    {
        static_assert(W == 4, "4 lanes per target");
        combine(lane_xor<2>(s), lane_xor<2>(c));
        combine(lane_xor<1>(s), lane_xor<1>(c));
    }
    __device__ void combine(T s2, T c2)
    {
        T t = s + s2;
        T bb = t - s;
        T err = (s - (t - bb)) + (s2 - bb);
        c = c + c2 - err;
        s = t;
    }
    __device__ double value() const { return (double)s - (double)c; }
};


// Per-target candidate lists for the 16 targets of a wavefront (targets
// 16 w + k, k = 0..15), built with G lanes per target (G = 16: sub-blocks of 4
// targets; G = 8: of 8): for each sub-block the wavefront lists the staged
// entries near the sub-block's box (box_ok(d2, Rs2, p): d2 the squared
// distance of entry p to the box, Rs the largest reach of the sub-block's
// targets; with FULL the entry is read as one vector, w included), then each
// target's G lanes keep the entries that accept(target position, reach, e).
// pos(k) and reach(k) give target slot k's position and reach (0: no list);
// every lane calls them.  sub is the wavefront's scratch list (room for
// subcap entries; a sub-block with more marks its targets' lists incomplete).
// Writes tls[(16 w + k) * cap ...] and tlen[16 w + k]; a length above cap
// means the list is incomplete and the caller must walk the staged set
// instead.
template <class T, bool FULL, int G, class Pos, class Reach, class BoxOk, class Accept>
__device__ inline void build_lists(int nstg, const vec4_t<T> *stg, uint16_t *sub, int subcap,
                                   uint16_t *tls, int cap, int *tlen, Pos pos, Reach reach,
                                   BoxOk box_ok, Accept accept)
{
    static_assert(G == 8 || G == 16, "8 or 16 lanes per target");
    constexpr int TPS = kWave / G;   // targets per sub-block
    constexpr int NSB = 16 / TPS;    // sub-blocks per wavefront
    const int w = wave_id(), lane = lane_id(), g = lane / G, j = lane % G;
    for (int sb = 0; sb < NSB; ++sb) {
        const int k = TPS * sb + g;  // this lane's target slot in the wave
        vec4_t<T> tp = pos(k);
        T rk = reach(k);
        T bigT = T(3.0e38);
        bool act = rk > T(0);
        T lox = wmin_lanes<G>(act ? tp.x : bigT), loy = wmin_lanes<G>(act ? tp.y : bigT),
          loz = wmin_lanes<G>(act ? tp.z : bigT);
        T hix = wmax_lanes<G>(act ? tp.x : -bigT), hiy = wmax_lanes<G>(act ? tp.y : -bigT),
          hiz = wmax_lanes<G>(act ? tp.z : -bigT);
        T Rs = wmax_lanes<G>(rk);
        int len = 0;
        if (Rs > T(0)) {
            T Rs2 = Rs * Rs;
            T bcx = T(0.5) * (lox + hix), bcy = T(0.5) * (loy + hiy), bcz = T(0.5) * (loz + hiz);
            T bex = T(0.5) * (hix - lox), bey = T(0.5) * (hiy - loy), bez = T(0.5) * (hiz - loz);
            int nsub = 0;
            wave_sync();
            for (int base = 0; base < nstg; base += kWave) {
                int idx = base + lane;
                bool hit = false;
                if (idx < nstg) {
                    // FULL: box_ok reads the w component too (one vector read)
                    const vec4_t<T> p = FULL ? lds_ld4<T>(&stg[idx]) : stg[idx];
                    hit = box_ok(pt_box_d2<T>(p.x, p.y, p.z, bcx, bcy, bcz, bex, bey, bez), Rs2, p);
                }
                uint64_t m = __ballot(hit);
                const int ps = nsub + __popcll(m & lanemask_lt());
                if (hit && ps < subcap) sub[ps] = (uint16_t)idx;
                nsub += __popcll(m);
            }
            wave_sync();
            if (nsub > subcap) {
                // the sub-block list did not fit: its targets walk the staged set
                if (j == 0) tlen[16 * w + k] = cap + 1;
                continue;
            }
            uint16_t *L = tls + (size_t)(16 * w + k) * cap;
            constexpr uint64_t gmask = G == 16 ? 0xffffull : 0xffull;
            for (int base = 0; base < nsub; base += G) {
                int k0 = base + j;
                bool hit = false;
                int e = 0;
                if (k0 < nsub && act) {
                    e = sub[k0];
                    hit = accept(tp, rk, e);
                }
                uint64_t m = __ballot(hit);
                uint32_t gm = (uint32_t)((m >> (G * g)) & gmask);
                int p = len + __popc(gm & ((1u << j) - 1u));
                if (hit && p < cap) L[p] = (uint16_t)e;
                len += __popc(gm);
            }
        }
        if (j == 0) tlen[16 * w + k] = len;
    }
    wave_sync();
}

}  // namespace apr
