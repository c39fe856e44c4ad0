// One split/merge pass (paper Sec. 2.2 splitting, Sec. 2.3 merging, Sec. 2.5
// order: split from the lowest level up, merge from the highest level down, a
// particle changes level at most once per pass).
//
// Split: a per-particle zone test and one scan place the new children, which
// are numbered in the order of their parents' ids (a radix sort of the
// splitting parents), so the result does not depend on the array order; the
// child axis, offset and the exact-centre-of-mass coordinate pair are
// computed in FP64 with no contraction, so positions match a plain FP64
// evaluation except for the last-place differences of sin/cos.
//
// Merge, per level l: the level-l candidates are compacted, sorted by id
// (stable radix sort), and paired by a k-d tree built level-synchronously over
// all nodes at once: per tree level, integer atomics give each node's extent,
// coordinate sum, count below the cut and the (coordinate, id)-extreme
// particles near the cut (integer atomics are order-independent, so the tree
// is deterministic), and a stable scan partitions every node.  The tree's
// rules (quantised coordinates, cut at floor(mean), even counts) are those in
// include/apr.h.  Finally the leaf pairs whose centre of mass leaves the
// level's zone merge, and a stable compaction removes the dropped particles.
#include "common.hpp"

namespace apr {

namespace {

constexpr int kMaxZones = 8;
constexpr double kCbrtHalf = 0.79370052598409973737585281963615;  // 2^(-1/3)
constexpr double kCbrtTwo = 1.2599210498948731647672106072782;    // 2^(1/3)
constexpr uint64_t kGamma = 0x9e3779b97f4a7c15ULL;
constexpr double kQuant = 2097152.0;  // 2^21 steps per axis
constexpr int kIdBits = 43;           // (coordinate, id) keys: 21 + 43 bits

struct Zones {
    int nz, bg, derefine;
    double c[kMaxZones][3];
    int nsh[kMaxZones];
    int cyl[kMaxZones];  // 1: cylinders along z through c (z left out)
    double r[kMaxZones][8];
    int ell[kMaxZones][8];
};

// z offset from zone k's centre as the zone's shape counts it
__device__ inline double zone_dz(const Zones &Z, int k, double z)
{
    return Z.cyl[k] ? 0.0 : z - Z.c[k][2];
}

// Level of a point: innermost sphere (or cylinder) of each zone (strict),
// combined by max (or min when derefining); *which = first zone giving the
// combined level.  shrink < 1 scales the radii (a conservative level near a
// boundary); 1 is the exact test.
__device__ int zone_level(const Zones &Z, double x, double y, double z, int *which,
                          double shrink = 1.0)
{
#pragma clang fp contract(off)
    int best = Z.bg, w = -1;
    for (int k = 0; k < Z.nz; ++k) {
        double dx = x - Z.c[k][0], dy = y - Z.c[k][1], dz = zone_dz(Z, k, z);
        double d2 = dx * dx + dy * dy + dz * dz;
        int lev = -1;
        for (int s = 0; s < Z.nsh[k]; ++s) {
            double rr = Z.r[k][s] * shrink;
            if (d2 < rr * rr) lev = Z.ell[k][s];
        }
        if (lev < 0) continue;
        if (Z.derefine ? (lev < best) : (lev > best)) {
            best = lev;
            w = k;
        } else if (lev == best && w < 0) {
            w = k;
        }
    }
    if (which) *which = w;
    return best;
}

// SplitMix64 (Steele, Lea & Flood 2014): k-th output from state s.
__device__ inline uint64_t sm64(uint64_t s, uint64_t k)
{
    uint64_t z = s + k * kGamma;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

__device__ inline uint64_t stream_state(uint64_t seed, int64_t step, int64_t id)
{
    uint64_t a = sm64((uint64_t)step, 1);
    uint64_t b = sm64((uint64_t)id ^ a, 1);
    return sm64(seed ^ b, 1);
}

__device__ inline double u53(uint64_t v) { return (double)(v >> 11) * 0x1.0p-53; }

// Split axis: tangential to zone `zone` (rotated about x - c, z left out for
// a cylinder zone, by 2 pi U1), or
// uniform on the sphere (cos theta = 2 U1 - 1, phi = 2 pi U2).
__device__ void split_axis(const Zones &Z, int zone, int mode, uint64_t s, double x, double y,
                           double z, double w[3])
{
#pragma clang fp contract(off)
    const double pi = 3.14159265358979323846;
    double U1 = u53(sm64(s, 1)), U2 = u53(sm64(s, 2));
    if (mode == APR_SPLIT_TANGENTIAL && zone >= 0) {
        double v[3] = {x - Z.c[zone][0], y - Z.c[zone][1], zone_dz(Z, zone, z)};
        double vn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        if (vn > 0.0) {
            int k = 0;
            if (fabs(v[1]) < fabs(v[k])) k = 1;
            if (fabs(v[2]) < fabs(v[k])) k = 2;
            double e[3] = {0.0, 0.0, 0.0};
            e[k] = 1.0;
            double w0[3] = {v[1] * e[2] - v[2] * e[1], v[2] * e[0] - v[0] * e[2],
                            v[0] * e[1] - v[1] * e[0]};
            double wn = sqrt(w0[0] * w0[0] + w0[1] * w0[1] + w0[2] * w0[2]);
            w0[0] /= wn;
            w0[1] /= wn;
            w0[2] /= wn;
            double vh[3] = {v[0] / vn, v[1] / vn, v[2] / vn};
            double b[3] = {vh[1] * w0[2] - vh[2] * w0[1], vh[2] * w0[0] - vh[0] * w0[2],
                           vh[0] * w0[1] - vh[1] * w0[0]};
            double t = 2.0 * pi * U1;
            double ct = cos(t), st = sin(t);
            for (int i = 0; i < 3; ++i) w[i] = w0[i] * ct + b[i] * st;
            return;
        }
    }
    double cth = 2.0 * U1 - 1.0;
    double sth = sqrt(fmax(0.0, 1.0 - cth * cth));
    double ph = 2.0 * pi * U2;
    w[0] = sth * cos(ph);
    w[1] = sth * sin(ph);
    w[2] = cth;
}

// Coordinates of the two children x +- d with x+ + x- = 2x exactly whenever
// |d| <= |x|: round the child on the far side from zero, take the exact shift
// d' = x_far - x, set the near child to x - d' (exact).
__device__ void split_pair_coord(double x, double d, double *xp, double *xm)
{
#pragma clang fp contract(off)
    if (x != 0.0 && fabs(d) <= fabs(x)) {
        double sgn = x > 0.0 ? 1.0 : -1.0;
        double far = x + sgn * fabs(d);
        double dd = far - x;
        double near = x - dd;
        bool plus_is_far = (d * sgn) >= 0.0;
        *xp = plus_is_far ? far : near;
        *xm = plus_is_far ? near : far;
    } else {
        *xp = x + d;
        *xm = x - d;
    }
}

__device__ inline double wrap(double v, const Box &b, int k)
{
    if (!b.periodic) return v;
    double hi = b.lo[k] + b.L[k];
    if (v >= hi) return v - b.L[k];
    if (v < b.lo[k]) return v + b.L[k];
    return v;
}

struct SArr {
    double *x, *y, *z, *vx, *vy, *vz, *u, *h, *ax, *ay, *az, *dudt;
    int8_t *level;
    int64_t *id;
};

__global__ void k_split_flags(int64_t n, SArr s, Zones Z, const uint8_t *active, uint32_t *flag,
                              int8_t *zone_of)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int w;
    int lz = zone_level(Z, s.x[i], s.y[i], s.z[i], &w);
    flag[i] = (s.level[i] < lz && (!active || active[i])) ? 1u : 0u;
    zone_of[i] = (int8_t)w;
}

template <class D>
__global__ void k_split_apply(int64_t n, SArr s, Zones Z, Box b, const uint32_t *flag,
                              const uint32_t *rank, const int8_t *zone_of, const D *dnn,
                              double r_sep_factor, double nn_cap, int mode, uint64_t seed,
                              int64_t step, int64_t next_id, const uint32_t *idrank,
                              uint8_t *changed, int64_t *origin)
{
#pragma clang fp contract(off)
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flag[i]) return;
    int64_t slot = n + rank[i];
    uint64_t st = stream_state(seed, step, s.id[i]);
    double w[3];
    double px = s.x[i], py = s.y[i], pz = s.z[i];
    split_axis(Z, zone_of[i], mode, st, px, py, pz, w);
    double r = r_sep_factor * s.h[i];
    if (nn_cap > 0.0 && dnn) {
        double dn = (double)dnn[i];
        if (isfinite(dn) && nn_cap * dn < r) r = nn_cap * dn;
    }
    double p[3] = {px, py, pz}, xp[3], xm[3];
    for (int k = 0; k < 3; ++k) split_pair_coord(p[k], r * w[k], &xp[k], &xm[k]);
    s.x[slot] = wrap(xm[0], b, 0);
    s.y[slot] = wrap(xm[1], b, 1);
    s.z[slot] = wrap(xm[2], b, 2);
    s.x[i] = wrap(xp[0], b, 0);
    s.y[i] = wrap(xp[1], b, 1);
    s.z[i] = wrap(xp[2], b, 2);
    s.vx[slot] = s.vx[i];
    s.vy[slot] = s.vy[i];
    s.vz[slot] = s.vz[i];
    s.u[slot] = s.u[i];
    if (s.ax) s.ax[slot] = s.ax[i];
    if (s.ay) s.ay[slot] = s.ay[i];
    if (s.az) s.az[slot] = s.az[i];
    if (s.dudt) s.dudt[slot] = s.dudt[i];
    double hc = s.h[i] * kCbrtHalf;
    s.h[i] = hc;
    s.h[slot] = hc;
    int8_t lv = (int8_t)(s.level[i] + 1);
    s.level[i] = lv;
    s.level[slot] = lv;
    s.id[slot] = next_id + (int64_t)idrank[i];
    changed[i] = 1;
    changed[slot] = 1;
    if (origin) origin[slot] = i;
}

__global__ void k_iota64(int64_t *p, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = i;
}

__global__ void k_fill_u8(uint8_t *p, uint8_t v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Combines a value over the 64 lanes of a wavefront (every lane gets the result).
template <class T, class F>
__device__ inline T wave_reduce(T v, F op)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = op(v, (T)__shfl_xor(v, o, 64));
    return v;
}

__device__ inline int32_t imin(int32_t a, int32_t b) { return a < b ? a : b; }
__device__ inline int32_t imax(int32_t a, int32_t b) { return a > b ? a : b; }

// Highest level present: a grid-stride pass (at most kMaxLevelBlocks
// workgroups), reduced within each workgroup, one atomic per workgroup (one
// per wavefront made a million particles wait on 16k atomics to one word).
constexpr int kMaxLevelBlocks = 1024;
__global__ __launch_bounds__(256) void k_max_level(int64_t n, const int8_t *level, int32_t *out)
{
    __shared__ int32_t red[256 / kWave];
    int32_t v = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        v = imax(v, (int32_t)level[i]);
    v = wave_reduce(v, imax);
    if (__lane_id() == 0) red[threadIdx.x / kWave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t m = red[0];
        for (int k = 1; k < 256 / kWave; ++k) m = imax(m, red[k]);
        atomicMax(out, m);
    }
}

// merge candidates of level l: not changed in this pass, not removed, and
// (individual timesteps) active; slots >= n0 are this pass's children
__global__ void k_cand_flags(int64_t n, const int8_t *level, const uint8_t *changed,
                             const uint8_t *removed, int l, const uint8_t *active, int64_t n0,
                             uint32_t *flag)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    flag[i] = (level[i] == l && !changed[i] && !removed[i] && (!active || i >= n0 || active[i]))
                  ? 1u
                  : 0u;
}

// Counts the merge candidates of level l that lie outside the level-l region
// of the zones, or within a relative 1e-9 of its boundary (*out, zeroed by the
// caller).  None, with zones whose level can only fall with the distance from
// one centre (merge_tree_skippable), means that no pair's centre of mass can
// lie outside it either: no pair merges and the pairing tree can be skipped.
__global__ void k_cand_outside(int64_t n, const uint32_t *flag, SArr s, Zones Z, int l,
                               uint32_t *out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flag[i]) return;
    if (zone_level(Z, s.x[i], s.y[i], s.z[i], nullptr, 1.0 - 1e-9) < l) atomicAdd(out, 1u);
}

__global__ void k_compact_idx(int64_t n, const uint32_t *flag, const uint32_t *pos,
                              uint32_t *out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && flag[i]) out[pos[i]] = (uint32_t)i;
}

__global__ void k_id_keys(int64_t m, const uint32_t *slot, const int64_t *id, int high,
                          uint32_t *key)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    uint64_t v = (uint64_t)id[slot[i]];
    key[i] = high ? (uint32_t)(v >> 32) : (uint32_t)v;
}

// idrank[slot[r]] = r: each listed slot's place in the sorted list
__global__ void k_rank_of(int64_t m, const uint32_t *slot, uint32_t *idrank)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < m) idrank[slot[r]] = (uint32_t)r;
}

__device__ inline int32_t quantise(double v, double lo, double s)
{
    double f = floor((v - lo) * s);
    if (f < 0.0) f = 0.0;
    if (f > kQuant - 1.0) f = kQuant - 1.0;
    return (int32_t)f;
}

// quantised coordinates, stored per particle slot
__global__ void k_quant(int64_t m, const uint32_t *slot, SArr s, Box b, double s0, double s1,
                        double s2, int32_t *qx, int32_t *qy, int32_t *qz)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    uint32_t p = slot[i];
    qx[p] = quantise(s.x[p], b.lo[0], s0);
    qy[p] = quantise(s.y[p], b.lo[1], s1);
    qz[p] = quantise(s.z[p], b.lo[2], s2);
}

// ------------------------------------------------------------ pairing tree
// Element arrays (position i in the tree order): es[i] particle slot, lo[i],
// hi[i] the range of its node.  Node statistics live at the node's start.
// A depth takes four passes: min / max and coordinate sums, counts about
// the cut, each element's side (then a scan of the sides), the partition,
// which also clears the next depth's nodes (their own array: a left child
// starts where its parent does, whose statistics the partition still reads).
struct Node {
    int32_t mn[3], mx[3];
    unsigned long long sum[3];
    uint32_t kc, keq;
    unsigned long long amin_c, amax_c, amin_c1, amax_c1;
    int32_t ax, kp;  // axis and left count, stored for the passes after the one that finds them
};

struct TreeArgs {
    int64_t m;
    const uint32_t *es;
    const int32_t *lo, *hi;
    const int32_t *q[3];
    const int64_t *id;
    Node *node;
};

__device__ inline bool active(const TreeArgs &a, int64_t i) { return a.hi[i] - a.lo[i] > 2; }

__device__ inline void clear_node(Node &nd)
{
    for (int k = 0; k < 3; ++k) {
        nd.mn[k] = INT32_MAX;
        nd.mx[k] = INT32_MIN;
        nd.sum[k] = 0;
    }
    nd.kc = 0;
    nd.keq = 0;
    nd.amin_c = ~0ull;
    nd.amax_c = 0;
    nd.amin_c1 = ~0ull;
    nd.amax_c1 = 0;
}

// True when every active lane of the wavefront works on the same node (the
// rule at the upper levels of the tree): the wavefront then combines its
// lanes first and one lane updates the node, instead of one atomic per
// element on a single address.  *first receives that lane.
__device__ inline bool wave_one_node(bool act, int32_t L, int *first)
{
    uint64_t m = __ballot(act);
    if (m == 0) return false;
    *first = __ffsll((unsigned long long)m) - 1;
    int32_t L0 = __shfl(L, *first, 64);
    return __all(!act || L == L0) != 0;
}

// Axis of the node's largest integer extent (ties to the lower axis), from
// its completed min / max.
__device__ inline int node_axis(const Node &nd)
{
    int ax = 0;
    for (int k = 1; k < 3; ++k)
        if (nd.mx[k] - nd.mn[k] > nd.mx[ax] - nd.mn[ax]) ax = k;
    return ax;
}

__device__ inline unsigned long long umin64(unsigned long long a, unsigned long long b)
{
    return a < b ? a : b;
}
__device__ inline unsigned long long umax64(unsigned long long a, unsigned long long b)
{
    return a > b ? a : b;
}
__device__ inline unsigned long long uadd64(unsigned long long a, unsigned long long b)
{
    return a + b;
}

__global__ void k_tree_minmax(TreeArgs a)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool act = i < a.m && active(a, i);
    int32_t L = act ? a.lo[i] : -1;
    uint32_t p = act ? a.es[i] : 0u;
    int first = 0;
    if (wave_one_node(act, L, &first)) {
        int32_t mn[3], mx[3];
        unsigned long long sm[3];
        for (int k = 0; k < 3; ++k) {
            int32_t v = act ? a.q[k][p] : 0;
            mn[k] = wave_reduce(act ? v : INT32_MAX, imin);
            mx[k] = wave_reduce(act ? v : INT32_MIN, imax);
            sm[k] = wave_reduce(act ? (unsigned long long)v : 0ull, uadd64);
        }
        if (__lane_id() == first) {
            Node &nd = a.node[L];
            for (int k = 0; k < 3; ++k) {
                atomicMin(&nd.mn[k], mn[k]);
                atomicMax(&nd.mx[k], mx[k]);
                atomicAdd(&nd.sum[k], sm[k]);
            }
        }
        return;
    }
    if (!act) return;
    Node &nd = a.node[L];
    for (int k = 0; k < 3; ++k) {
        atomicMin(&nd.mn[k], a.q[k][p]);
        atomicMax(&nd.mx[k], a.q[k][p]);
        atomicAdd(&nd.sum[k], (unsigned long long)a.q[k][p]);
    }
}

__global__ void k_tree_count(TreeArgs a)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool act = i < a.m && active(a, i);
    int32_t L = act ? a.lo[i] : -1;
    int first = 0;
    bool lt = false, eq = false;
    unsigned long long key = 0;
    if (act) {
        Node &nd = a.node[L];
        // the axis from the completed min / max; the node's first element
        // stores it for the later passes (no element reads it here)
        const int ax = node_axis(nd);
        if (i == L) nd.ax = ax;
        int64_t n = a.hi[i] - L;
        int64_t c = (int64_t)(nd.sum[ax] / (unsigned long long)n);
        uint32_t p = a.es[i];
        int64_t v = a.q[ax][p];
        key = ((unsigned long long)v << kIdBits) |
              ((unsigned long long)a.id[p] & ((1ull << kIdBits) - 1));
        lt = v < c;
        eq = v == c;
    }
    if (wave_one_node(act, L, &first)) {
        uint32_t kc = (uint32_t)__popcll(__ballot(act && lt));
        uint32_t keq = (uint32_t)__popcll(__ballot(act && eq));
        unsigned long long amax_c = wave_reduce((act && lt) ? key : 0ull, umax64);
        unsigned long long amin_c = wave_reduce((act && !lt) ? key : ~0ull, umin64);
        unsigned long long amax_c1 = wave_reduce((act && (lt || eq)) ? key : 0ull, umax64);
        unsigned long long amin_c1 = wave_reduce((act && !(lt || eq)) ? key : ~0ull, umin64);
        if (__lane_id() == first) {
            Node &nd = a.node[L];
            if (kc) atomicAdd(&nd.kc, kc);
            if (keq) atomicAdd(&nd.keq, keq);
            atomicMax(&nd.amax_c, amax_c);
            atomicMin(&nd.amin_c, amin_c);
            atomicMax(&nd.amax_c1, amax_c1);
            atomicMin(&nd.amin_c1, amin_c1);
        }
        return;
    }
    if (!act) return;
    Node &nd = a.node[L];
    if (lt) {
        atomicAdd(&nd.kc, 1u);
        atomicMax(&nd.amax_c, key);
    } else {
        atomicMin(&nd.amin_c, key);
    }
    if (eq) atomicAdd(&nd.keq, 1u);
    if (lt || eq) atomicMax(&nd.amax_c1, key);
    else atomicMin(&nd.amin_c1, key);
}

// The node's cut from its completed statistics: the centroid c (floor of the
// integer mean) with kc elements below it, moved up one step when none is;
// kp elements go left.  An odd kc moves the element nearest the plane (by
// (coordinate, id)) from the larger side; all-equal coordinates split by
// position.
struct Cut {
    int32_t cut, kp, all_eq;
    unsigned long long moved;
};

__device__ inline Cut node_cut(const Node &nd, int64_t n)
{
    Cut r;
    int64_t c = (int64_t)(nd.sum[nd.ax] / (unsigned long long)n);
    int64_t k = nd.kc;
    unsigned long long amin = nd.amin_c, amax = nd.amax_c;
    if (k == 0) {  // nothing below the cut: move it up one step
        c += 1;
        k = nd.keq;
        amin = nd.amin_c1;
        amax = nd.amax_c1;
    }
    r.cut = (int32_t)c;
    r.all_eq = 0;
    r.moved = ~0ull;
    if (k == n) {
        r.all_eq = 1;
        r.kp = (int32_t)(2 * (n / 4));
    } else if (k % 2 == 0) {
        r.kp = (int32_t)k;
    } else if (k < n - k) {
        r.kp = (int32_t)(k + 1);
        r.moved = amin;
    } else {
        r.kp = (int32_t)(k - 1);
        r.moved = amax;
    }
    return r;
}

// Side of every element.  Each takes the node's cut itself; the node's first
// element stores kp for the partition (no element reads it here).
__global__ void k_tree_left(TreeArgs a, uint32_t *left, int32_t *more)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *more = 0;  // the partition after this pass sets it
    if (i >= a.m) return;
    if (!active(a, i)) {
        left[i] = 1u;  // leaves stay in place
        return;
    }
    int32_t L = a.lo[i];
    const Cut cu = node_cut(a.node[L], a.hi[i] - L);
    if (i == L) a.node[L].kp = cu.kp;
    uint32_t p = a.es[i];
    bool l;
    if (cu.all_eq) {
        l = (i - L) < cu.kp;
    } else {
        int64_t v = a.q[a.node[L].ax][p];
        l = v < cu.cut;
        unsigned long long key = ((unsigned long long)v << kIdBits) |
                                 ((unsigned long long)a.id[p] & ((1ull << kIdBits) - 1));
        if (key == cu.moved) l = !l;
    }
    left[i] = l ? 1u : 0u;
}

__global__ void k_tree_partition(TreeArgs a, const uint32_t *left, const uint32_t *lscan,
                                 uint32_t *es2, int32_t *lo2, int32_t *hi2, int32_t *more,
                                 Node *next)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.m) return;
    int32_t L = a.lo[i], H = a.hi[i];
    if (H - L <= 2) {
        es2[i] = a.es[i];
        lo2[i] = L;
        hi2[i] = H;
        return;
    }
    int32_t kp = a.node[L].kp;
    int64_t lr = (int64_t)lscan[i] - (int64_t)lscan[L];
    int64_t pos;
    int32_t nl, nh;
    if (left[i]) {
        pos = L + lr;
        nl = L;
        nh = L + kp;
    } else {
        pos = L + kp + (i - L - lr);
        nl = L + kp;
        nh = H;
    }
    es2[pos] = a.es[i];
    lo2[pos] = nl;
    hi2[pos] = nh;
    if (nh - nl > 2) {
        if (pos == nl) clear_node(next[nl]);  // one element per child starts it
        atomicOr(more, 1);
    }
}

// A tree of at most kSmallTree elements (the candidates of an
// individual-timestep substep, or of a step's pass away from the zones'
// edges) in one workgroup: every depth of the level-synchronous construction
// above, with the same statistics, cut and stable partition, runs in LDS
// (gfx950 gives a workgroup up to 160 KB), one element per thread, until no
// node holds more than two elements.  One launch instead of five per depth,
// and no host check between depths.  A wavefront whose active elements share
// a node combines them before one lane updates it, as the kernels above do.
// es_out receives the final order (pairs adjacent).
constexpr int kSmallTree = 1024;

__global__ __launch_bounds__(kSmallTree) void k_tree_small(int32_t m, const uint32_t *cand,
                                                           const int32_t *q0, const int32_t *q1,
                                                           const int32_t *q2, const int64_t *id,
                                                           uint32_t *es_out)
{
    __shared__ uint32_t es[2][kSmallTree];
    __shared__ int32_t lo[2][kSmallTree], hi[2][kSmallTree];
    __shared__ Node nd[kSmallTree];
    __shared__ uint32_t sc[kSmallTree], ex[kSmallTree];
    __shared__ int s_more;
    const int i = threadIdx.x, lane = __lane_id();
    const int32_t *q[3] = {q0, q1, q2};
    if (i < m) {
        es[0][i] = cand[i];
        lo[0][i] = 0;
        hi[0][i] = m;
    }
    int cur = 0;
    bool more = m > 2;
    // m is even, so every node is: each depth splits every node of four or
    // more elements into two non-empty even parts, and m / 2 depths bound
    // the loop
    for (int depth = 0; more && depth < kSmallTree / 2; ++depth) {
        if (i < m) clear_node(nd[i]);
        __syncthreads();
        const bool act = i < m && hi[cur][i] - lo[cur][i] > 2;
        const int32_t L = act ? lo[cur][i] : -1, H = act ? hi[cur][i] : 0;
        const uint32_t p = act ? es[cur][i] : 0u;
        // min / max and coordinate sums of each node
        int first = 0;
        if (wave_one_node(act, L, &first)) {
            int32_t mn[3], mx[3];
            unsigned long long sm[3];
            for (int k = 0; k < 3; ++k) {
                const int32_t v = act ? q[k][p] : 0;
                mn[k] = wave_reduce(act ? v : INT32_MAX, imin);
                mx[k] = wave_reduce(act ? v : INT32_MIN, imax);
                sm[k] = wave_reduce(act ? (unsigned long long)v : 0ull, uadd64);
            }
            if (lane == first) {
                Node &n0 = nd[L];
                for (int k = 0; k < 3; ++k) {
                    atomicMin(&n0.mn[k], mn[k]);
                    atomicMax(&n0.mx[k], mx[k]);
                    atomicAdd(&n0.sum[k], sm[k]);
                }
            }
        } else if (act) {
            for (int k = 0; k < 3; ++k) {
                atomicMin(&nd[L].mn[k], q[k][p]);
                atomicMax(&nd[L].mx[k], q[k][p]);
                atomicAdd(&nd[L].sum[k], (unsigned long long)q[k][p]);
            }
        }
        __syncthreads();
        // counts and extreme keys about the centroid on the widest axis
        bool lt = false, eq = false;
        unsigned long long key = 0;
        if (act) {
            const int ax = node_axis(nd[L]);
            if (i == L) nd[L].ax = ax;
            const int64_t c = (int64_t)(nd[L].sum[ax] / (unsigned long long)(H - L));
            const int64_t v = q[ax][p];
            key = ((unsigned long long)v << kIdBits) |
                  ((unsigned long long)id[p] & ((1ull << kIdBits) - 1));
            lt = v < c;
            eq = v == c;
        }
        if (wave_one_node(act, L, &first)) {
            const uint32_t kc = (uint32_t)__popcll(__ballot(act && lt));
            const uint32_t keq = (uint32_t)__popcll(__ballot(act && eq));
            const unsigned long long amax_c = wave_reduce((act && lt) ? key : 0ull, umax64);
            const unsigned long long amin_c = wave_reduce((act && !lt) ? key : ~0ull, umin64);
            const unsigned long long amax_c1 =
                wave_reduce((act && (lt || eq)) ? key : 0ull, umax64);
            const unsigned long long amin_c1 =
                wave_reduce((act && !(lt || eq)) ? key : ~0ull, umin64);
            if (lane == first) {
                Node &n0 = nd[L];
                if (kc) atomicAdd(&n0.kc, kc);
                if (keq) atomicAdd(&n0.keq, keq);
                atomicMax(&n0.amax_c, amax_c);
                atomicMin(&n0.amin_c, amin_c);
                atomicMax(&n0.amax_c1, amax_c1);
                atomicMin(&n0.amin_c1, amin_c1);
            }
        } else if (act) {
            if (lt) {
                atomicAdd(&nd[L].kc, 1u);
                atomicMax(&nd[L].amax_c, key);
            } else {
                atomicMin(&nd[L].amin_c, key);
            }
            if (eq) atomicAdd(&nd[L].keq, 1u);
            if (lt || eq) atomicMax(&nd[L].amax_c1, key);
            else atomicMin(&nd[L].amin_c1, key);
        }
        __syncthreads();
        // each element's side (elements of finished nodes count as left and
        // stay in place)
        uint32_t left = 1u;
        int32_t kp = 0;
        if (act) {
            const Cut cu = node_cut(nd[L], H - L);
            kp = cu.kp;
            if (cu.all_eq) {
                left = (i - L) < cu.kp ? 1u : 0u;
            } else {
                const int64_t v = q[nd[L].ax][p];
                bool l = v < cu.cut;
                const unsigned long long k2 = ((unsigned long long)v << kIdBits) |
                                              ((unsigned long long)id[p] & ((1ull << kIdBits) - 1));
                if (k2 == cu.moved) l = !l;
                left = l ? 1u : 0u;
            }
        }
        // exclusive scan of the sides over the elements (inclusive in sc,
        // then each element's exclusive value in ex)
        sc[i] = i < m ? left : 0u;
        __syncthreads();
        for (int off = 1; off < kSmallTree; off <<= 1) {
            const uint32_t u = i >= off ? sc[i - off] : 0u;
            __syncthreads();
            sc[i] += u;
            __syncthreads();
        }
        ex[i] = sc[i] - (i < m ? left : 0u);
        if (i == 0) s_more = 0;
        __syncthreads();
        // stable partition of every active node into [L, L + kp) and
        // [L + kp, H); finished nodes keep their place
        const int nx = 1 - cur;
        if (i < m) {
            if (!act) {
                es[nx][i] = es[cur][i];
                lo[nx][i] = lo[cur][i];
                hi[nx][i] = hi[cur][i];
            } else {
                const int32_t lr = (int32_t)(ex[i] - ex[L]);
                int32_t pos, nl, nh;
                if (left) {
                    pos = L + lr;
                    nl = L;
                    nh = L + kp;
                } else {
                    pos = L + kp + (i - L - lr);
                    nl = L + kp;
                    nh = H;
                }
                es[nx][pos] = p;
                lo[nx][pos] = nl;
                hi[nx][pos] = nh;
                if (nh - nl > 2) s_more = 1;
            }
        }
        __syncthreads();
        cur = nx;
        more = s_more != 0;
        __syncthreads();  // s_more and the node statistics are rewritten next
    }
    if (i < m) es_out[i] = es[cur][i];
}

__global__ void k_tree_root(int64_t m, int32_t *lo, int32_t *hi, Node *node)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    lo[i] = 0;
    hi[i] = (int32_t)m;
    if (i == 0 && m > 2) clear_node(node[0]);
}

// Centre of mass of a merging pair along axis k (equal masses, Sec. 2.3).
// Periodic boxes: the removed particle's coordinate o is taken at its minimum
// image about the kept one's, c, and the mean wrapped back into the box, so a
// pair across the boundary merges beside it, not at mid-box.  A pair closer
// than half the box averages as it is.
__device__ inline double merge_mid(double c, double o, const Box &b, int k)
{
#pragma clang fp contract(off)
    if (b.periodic) {
        double d = o - c;
        if (d > 0.5 * b.L[k]) o -= b.L[k];
        else if (d < -0.5 * b.L[k]) o += b.L[k];
    }
    return wrap((c + o) * 0.5, b, k);
}

__global__ void k_merge_pairs(int64_t npairs, const uint32_t *es, SArr s, Zones Z, Box b, int l,
                              uint8_t *changed, uint8_t *removed, unsigned long long *count)
{
#pragma clang fp contract(off)
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= npairs) return;
    uint32_t p = es[2 * k], q = es[2 * k + 1];
    uint32_t keep = s.id[p] < s.id[q] ? p : q;
    uint32_t gone = keep == p ? q : p;
    double cx = merge_mid(s.x[keep], s.x[gone], b, 0);
    double cy = merge_mid(s.y[keep], s.y[gone], b, 1);
    double cz = merge_mid(s.z[keep], s.z[gone], b, 2);
    if (!(zone_level(Z, cx, cy, cz, nullptr) < l)) return;
    s.x[keep] = cx;
    s.y[keep] = cy;
    s.z[keep] = cz;
    s.vx[keep] = (s.vx[p] + s.vx[q]) * 0.5;
    s.vy[keep] = (s.vy[p] + s.vy[q]) * 0.5;
    s.vz[keep] = (s.vz[p] + s.vz[q]) * 0.5;
    s.u[keep] = (s.u[p] + s.u[q]) * 0.5;
    s.h[keep] = s.h[keep] * kCbrtTwo;
    s.level[keep] = (int8_t)(l - 1);
    changed[keep] = 1;
    removed[gone] = 1;
    atomicAdd(count, 1ull);
}

__global__ void k_keep_flags(int64_t n, const uint8_t *removed, uint32_t *flag)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = removed[i] ? 0u : 1u;
}

struct CompactArgs {
    double *d[12], *dt[12];
    int nd;
    int8_t *lev, *levt;
    int64_t *id, *idt;
    int64_t *org, *orgt;   // optional: slots before the pass
    uint8_t *chg, *chgt;   // the pass's changed flags (kept for the caller)
    const uint32_t *keep, *pos;
    int64_t n;
};

__global__ void k_compact_gather(CompactArgs a)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n || !a.keep[i]) return;
    uint32_t j = a.pos[i];
    for (int k = 0; k < a.nd; ++k) a.dt[k][j] = a.d[k][i];
    a.levt[j] = a.lev[i];
    a.idt[j] = a.id[i];
    if (a.org) a.orgt[j] = a.org[i];
    a.chgt[j] = a.chg[i];
}

__global__ void k_compact_back(CompactArgs a, int64_t m)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    for (int k = 0; k < a.nd; ++k) a.d[k][i] = a.dt[k][i];
    a.lev[i] = a.levt[i];
    a.id[i] = a.idt[i];
    if (a.org) a.org[i] = a.orgt[i];
    a.chg[i] = a.chgt[i];
}

unsigned grid(int64_t n) { return (unsigned)ceil_div(n > 0 ? n : 1, 256); }

// slot[0..m) into ascending id order: a stable LSD radix sort on the low 32
// bits of the id, then on the high 32 when ids reach that far.  Every id is
// below next_id, so the low-word sort needs only next_id's bit length.
// At most kSmallSort slots in one workgroup: each slot's place is the number
// of listed slots with a smaller id (the ids are unique, so the places are a
// permutation, the order any sort by id gives).
constexpr int kSmallSort = 1024;

__global__ __launch_bounds__(kSmallSort) void k_sort_small(int32_t m, uint32_t *slot,
                                                           const int64_t *id)
{
    __shared__ int64_t sid[kSmallSort];
    const int i = threadIdx.x;
    uint32_t p = 0;
    int64_t v = 0;
    if (i < m) {
        p = slot[i];
        v = id[p];
        sid[i] = v;
    }
    __syncthreads();
    int rank = 0;
    if (i < m)
        for (int k = 0; k < m; ++k) rank += sid[k] < v ? 1 : 0;
    __syncthreads();  // every thread has read its slot before any is overwritten
    if (i < m) slot[rank] = p;
}

int sort_slots_by_id(apr_ctx *c, uint32_t *slot, uint32_t *keys, int64_t m, const int64_t *id,
                     int64_t next_id)
{
    if (m <= 1) return APR_OK;
    if (m <= kSmallSort) {
        hipLaunchKernelGGL(k_sort_small, dim3(1), dim3(kSmallSort), 0, c->stream, (int32_t)m,
                           slot, id);
        APR_LAUNCHED(c);
        return APR_OK;
    }
    const bool high_ids = next_id > (int64_t)0xffffffffLL;
    int id_bits = 32;
    if (!high_ids) {
        id_bits = 1;
        while (id_bits < 32 && (((int64_t)1 << id_bits) < next_id)) ++id_bits;
    }
    hipLaunchKernelGGL(k_id_keys, dim3(grid(m)), dim3(256), 0, c->stream, m, slot, id, 0, keys);
    APR_LAUNCHED(c);
    int rc = radix_sort_u32(c, keys, slot, m, id_bits);
    if (rc || !high_ids) return rc;
    hipLaunchKernelGGL(k_id_keys, dim3(grid(m)), dim3(256), 0, c->stream, m, slot, id, 1, keys);
    APR_LAUNCHED(c);
    return radix_sort_u32(c, keys, slot, m, 32);
}

}  // namespace

// Whether the pairing tree of a level may be skipped when all its candidates
// lie inside that level's region (k_cand_outside): one zone in a
// non-periodic box whose levels never fall inward (and none below the
// background), combined by max.  Its level then falls with the distance from
// the centre (or the axis), and a pair's centre of mass is no farther out
// than the farther of the two: no pair of particles inside the level-l
// region can have its centre of mass outside it.  Exact: the oracle builds
// the tree and merges nothing either.
static bool merge_tree_skippable(const Zones &Z, const apr_params &P)
{
    if (Z.nz != 1 || Z.derefine || P.periodic) return false;
    if (Z.nsh[0] < 1 || Z.ell[0][0] < Z.bg) return false;
    for (int s = 1; s < Z.nsh[0]; ++s)
        if (Z.ell[0][s] < Z.ell[0][s - 1] || !(Z.r[0][s] < Z.r[0][s - 1])) return false;
    return true;
}

int split_merge(apr_ctx *c, apr_state *s, const apr_zone *zones, int nzones, int64_t step,
                int flags, int64_t *n_split, int64_t *n_merged, int64_t *n_spare,
                const uint8_t *active, int64_t *origin, uint8_t *made)
{
    const apr_params &P = c->p;
    if (nzones > kMaxZones) return fail(c, APR_ERR_INVALID, "at most 8 zones");
    bool do_split = flags == 0 || (flags & 1);
    bool do_merge = flags == 0 || (flags & 2);
    *n_split = 0;
    *n_merged = 0;
    *n_spare = 0;
    Zones Z;
    std::memset(&Z, 0, sizeof(Z));
    Z.nz = nzones;
    Z.bg = P.ell_background;
    Z.derefine = P.derefine;
    for (int k = 0; k < nzones; ++k) {
        for (int d = 0; d < 3; ++d) Z.c[k][d] = zones[k].c[d];
        if (zones[k].shape != APR_ZONE_SPHERE && zones[k].shape != APR_ZONE_CYLINDER)
            return fail(c, APR_ERR_INVALID, "zone shape");
        Z.cyl[k] = zones[k].shape == APR_ZONE_CYLINDER;
        Z.nsh[k] = zones[k].n;
        for (int sh = 0; sh < zones[k].n; ++sh) {
            Z.r[k][sh] = zones[k].r[sh];
            Z.ell[k][sh] = zones[k].ell[sh];
        }
    }
    if (s->next_id + s->n >= (int64_t)1 << kIdBits) return fail(c, APR_ERR_INVALID, "ids too large");
    Box b = make_box(P);
    SArr A = {s->x, s->y, s->z, s->vx, s->vy, s->vz, s->u, s->h,
              s->ax, s->ay, s->az, s->dudt, s->level, s->id};
    int64_t cap = s->capacity;
    int64_t n = s->n;
    int tok = prof_begin(c, APR_PROF_SPLITMERGE);

    uint32_t *flag = wsa<uint32_t>(c, "sm_flag", (size_t)cap);
    uint32_t *scan = wsa<uint32_t>(c, "sm_scan", (size_t)cap);
    uint32_t *tot = wsa<uint32_t>(c, "sm_tot", 4);
    int8_t *zone_of = wsa<int8_t>(c, "sm_zone", (size_t)cap);
    uint8_t *changed = wsa<uint8_t>(c, "sm_changed", (size_t)cap);
    uint8_t *removed = wsa<uint8_t>(c, "sm_removed", (size_t)cap);
    int32_t *imax = wsa<int32_t>(c, "sm_imax", 4);
    unsigned long long *mcount = wsa<unsigned long long>(c, "sm_mcount", 2);
    if (!flag || !scan || !tot || !zone_of || !changed || !removed || !imax || !mcount)
        return fail(c, APR_ERR_HIP, "split/merge workspace");
    hipLaunchKernelGGL(k_fill_u8, dim3(grid(cap)), dim3(256), 0, c->stream, changed, (uint8_t)0,
                       cap);
    hipLaunchKernelGGL(k_fill_u8, dim3(grid(cap)), dim3(256), 0, c->stream, removed, (uint8_t)0,
                       cap);
    if (origin)
        hipLaunchKernelGGL(k_iota64, dim3(grid(n)), dim3(256), 0, c->stream, origin, n);
    APR_LAUNCHED(c);
    const int64_t n0 = n;
    uint32_t h32 = 0;

    if (do_split) {
        hipLaunchKernelGGL(k_split_flags, dim3(grid(n)), dim3(256), 0, c->stream, n, A, Z, active,
                           flag, zone_of);
        APR_LAUNCHED(c);
        int rc = exclusive_scan_u32(c, flag, scan, n, tot);
        if (rc) return rc;
        APR_HIP(c, hipMemcpyAsync(&h32, tot, 4, hipMemcpyDeviceToHost, c->stream));
        APR_HIP(c, hipStreamSynchronize(c->stream));
        int64_t ns = h32;
        if (n + ns > cap) {
            prof_end(c, tok);
            *n_split = n + ns;
            return fail(c, APR_ERR_CAPACITY, "splits need more capacity");
        }
        if (ns > 0) {
            bool cap_nn = P.nn_cap > 0.0;
            if (cap_nn && c->dens_n != n) {
                prof_end(c, tok);
                return fail(c, APR_ERR_INVALID,
                            "nn_cap > 0 needs apr_density on the current state first");
            }
            // the children are numbered in the order of their parents' ids
            uint32_t *pslot = wsa<uint32_t>(c, "sm_cand", (size_t)n);
            uint32_t *pkey = wsa<uint32_t>(c, "sm_keys", (size_t)n);
            uint32_t *idrank = wsa<uint32_t>(c, "sm_idrank", (size_t)n);
            if (!pslot || !pkey || !idrank) return fail(c, APR_ERR_HIP, "split workspace");
            hipLaunchKernelGGL(k_compact_idx, dim3(grid(n)), dim3(256), 0, c->stream, n, flag,
                               scan, pslot);
            APR_LAUNCHED(c);
            rc = sort_slots_by_id(c, pslot, pkey, ns, s->id, s->next_id);
            if (rc) return rc;
            hipLaunchKernelGGL(k_rank_of, dim3(grid(ns)), dim3(256), 0, c->stream, ns, pslot,
                               idrank);
            APR_LAUNCHED(c);
            // the nearest-neighbour distances of the n parents, as the last
            // density pass wrote them: asked for by n, not by the capacity, so
            // that a capacity grown since then cannot reallocate (and lose) them
            if (P.precision == APR_FP32) {
                const float *dnn = cap_nn ? wsa<float>(c, "dnn32", (size_t)n) : nullptr;
                hipLaunchKernelGGL(k_split_apply<float>, dim3(grid(n)), dim3(256), 0, c->stream,
                                   n, A, Z, b, flag, scan, zone_of, dnn, P.r_sep_factor,
                                   P.nn_cap, P.split_mode, P.seed, step, s->next_id, idrank,
                                   changed, origin);
            } else {
                const double *dnn = cap_nn ? wsa<double>(c, "dnn64", (size_t)n) : nullptr;
                hipLaunchKernelGGL(k_split_apply<double>, dim3(grid(n)), dim3(256), 0, c->stream,
                                   n, A, Z, b, flag, scan, zone_of, dnn, P.r_sep_factor,
                                   P.nn_cap, P.split_mode, P.seed, step, s->next_id, idrank,
                                   changed, origin);
            }
            APR_LAUNCHED(c);
            n += ns;
            s->next_id += ns;
            s->n = n;
        }
        *n_split = ns;
    }

    if (do_merge && n > 1) {
        APR_HIP(c, hipMemsetAsync(imax, 0, 4, c->stream));
        APR_HIP(c, hipMemsetAsync(mcount, 0, 8, c->stream));
        hipLaunchKernelGGL(k_max_level, dim3(std::min<unsigned>(grid(n), kMaxLevelBlocks)),
                           dim3(256), 0, c->stream, n, s->level, imax);
        APR_LAUNCHED(c);
        int32_t lmax = 0;
        APR_HIP(c, hipMemcpyAsync(&lmax, imax, 4, hipMemcpyDeviceToHost, c->stream));
        APR_HIP(c, hipStreamSynchronize(c->stream));
        uint32_t *cand = wsa<uint32_t>(c, "sm_cand", (size_t)n);
        uint32_t *keys = wsa<uint32_t>(c, "sm_keys", (size_t)n);
        int32_t *q[3] = {wsa<int32_t>(c, "sm_qx", (size_t)n), wsa<int32_t>(c, "sm_qy", (size_t)n),
                         wsa<int32_t>(c, "sm_qz", (size_t)n)};
        uint32_t *es[2] = {wsa<uint32_t>(c, "sm_es0", (size_t)n),
                           wsa<uint32_t>(c, "sm_es1", (size_t)n)};
        int32_t *lo[2] = {wsa<int32_t>(c, "sm_lo0", (size_t)n), wsa<int32_t>(c, "sm_lo1", (size_t)n)};
        int32_t *hi[2] = {wsa<int32_t>(c, "sm_hi0", (size_t)n), wsa<int32_t>(c, "sm_hi1", (size_t)n)};
        Node *node[2] = {wsa<Node>(c, "sm_node0", (size_t)n), wsa<Node>(c, "sm_node1", (size_t)n)};
        int32_t *more = imax + 1;
        if (!cand || !keys || !q[2] || !es[1] || !lo[1] || !hi[1] || !node[0] || !node[1])
            return fail(c, APR_ERR_HIP, "merge workspace");
        double sc[3];
        for (int k = 0; k < 3; ++k) sc[k] = kQuant / b.L[k];
        const bool skippable = merge_tree_skippable(Z, P);
        for (int l = lmax; l >= 1; --l) {
            hipLaunchKernelGGL(k_cand_flags, dim3(grid(n)), dim3(256), 0, c->stream, n, s->level,
                               changed, removed, l, active, n0, flag);
            APR_LAUNCHED(c);
            int rc = exclusive_scan_u32(c, flag, scan, n, tot);
            if (rc) return rc;
            uint32_t hc[2] = {0, 0};
            if (skippable) {
                rc = fill_u32(c, tot + 2, 0u, 1);
                if (rc) return rc;
                hipLaunchKernelGGL(k_cand_outside, dim3(grid(n)), dim3(256), 0, c->stream, n,
                                   flag, A, Z, l, tot + 2);
                APR_LAUNCHED(c);
            }
            APR_HIP(c, hipMemcpyAsync(&hc[0], tot, 4, hipMemcpyDeviceToHost, c->stream));
            if (skippable)
                APR_HIP(c, hipMemcpyAsync(&hc[1], tot + 2, 4, hipMemcpyDeviceToHost, c->stream));
            APR_HIP(c, hipStreamSynchronize(c->stream));
            int64_t nc = hc[0];
            if (nc % 2) *n_spare += 1;
            int64_t m = nc - (nc % 2);
            if (m < 2) continue;
            if (skippable && hc[1] == 0) continue;  // no pair can merge at this level
            hipLaunchKernelGGL(k_compact_idx, dim3(grid(n)), dim3(256), 0, c->stream, n, flag,
                               scan, cand);
            rc = sort_slots_by_id(c, cand, keys, nc, s->id, s->next_id);
            if (rc) return rc;
            // the highest id (last) sits out when nc is odd; tree over the first m
            hipLaunchKernelGGL(k_quant, dim3(grid(m)), dim3(256), 0, c->stream, m, cand, A, b,
                               sc[0], sc[1], sc[2], q[0], q[1], q[2]);
            if (m <= kSmallTree) {
                // the whole tree in one workgroup, no host check between depths
                hipLaunchKernelGGL(k_tree_small, dim3(1), dim3(kSmallTree), 0, c->stream,
                                   (int32_t)m, cand, q[0], q[1], q[2], s->id, es[0]);
                APR_LAUNCHED(c);
                hipLaunchKernelGGL(k_merge_pairs, dim3(grid(m / 2)), dim3(256), 0, c->stream,
                                   m / 2, es[0], A, Z, b, l, changed, removed, mcount);
                APR_LAUNCHED(c);
                continue;
            }
            APR_HIP(c, hipMemcpyAsync(es[0], cand, (size_t)m * 4, hipMemcpyDeviceToDevice,
                                      c->stream));
            hipLaunchKernelGGL(k_tree_root, dim3(grid(m)), dim3(256), 0, c->stream, m, lo[0],
                               hi[0], node[0]);
            APR_LAUNCHED(c);
            // Depths run in batches between host checks of `more` (set by
            // the last partition when a node still holds more than two
            // elements): first about log2 m + 2 of them (a balanced tree's
            // depth), then 4 at a time.  A depth after the tree is complete
            // changes nothing: no node is active, so every element keeps its
            // place.
            int cur = 0;
            int depth = 0, batch = 2;
            for (int64_t mm = m; mm > 1; mm >>= 1) ++batch;
            while (m > 2) {
                for (int b2 = 0; b2 < batch; ++b2, ++depth) {
                    TreeArgs ta;
                    ta.m = m;
                    ta.es = es[cur];
                    ta.lo = lo[cur];
                    ta.hi = hi[cur];
                    for (int k = 0; k < 3; ++k) ta.q[k] = q[k];
                    ta.id = s->id;
                    ta.node = node[cur];
                    unsigned g = grid(m);
                    hipLaunchKernelGGL(k_tree_minmax, dim3(g), dim3(256), 0, c->stream, ta);
                    hipLaunchKernelGGL(k_tree_count, dim3(g), dim3(256), 0, c->stream, ta);
                    hipLaunchKernelGGL(k_tree_left, dim3(g), dim3(256), 0, c->stream, ta, flag,
                                       more);
                    APR_LAUNCHED(c);
                    rc = exclusive_scan_u32(c, flag, scan, m, nullptr);
                    if (rc) return rc;
                    hipLaunchKernelGGL(k_tree_partition, dim3(g), dim3(256), 0, c->stream, ta,
                                       flag, scan, es[1 - cur], lo[1 - cur], hi[1 - cur], more,
                                       node[1 - cur]);
                    APR_LAUNCHED(c);
                    cur = 1 - cur;
                }
                int32_t hm = 0;
                APR_HIP(c, hipMemcpyAsync(&hm, more, 4, hipMemcpyDeviceToHost, c->stream));
                APR_HIP(c, hipStreamSynchronize(c->stream));
                if (!hm) break;
                if (depth >= 4096) {
                    prof_end(c, tok);
                    return fail(c, APR_ERR_INVALID, "pairing tree deeper than 4096 levels");
                }
                batch = 4;
            }
            hipLaunchKernelGGL(k_merge_pairs, dim3(grid(m / 2)), dim3(256), 0, c->stream, m / 2,
                               es[cur], A, Z, b, l, changed, removed, mcount);
            APR_LAUNCHED(c);
        }
        unsigned long long nm = 0;
        APR_HIP(c, hipMemcpyAsync(&nm, mcount, 8, hipMemcpyDeviceToHost, c->stream));
        APR_HIP(c, hipStreamSynchronize(c->stream));
        *n_merged = (int64_t)nm;
        if (nm > 0) {
            // stable compaction of the survivors
            hipLaunchKernelGGL(k_keep_flags, dim3(grid(n)), dim3(256), 0, c->stream, n, removed,
                               flag);
            APR_LAUNCHED(c);
            int rc = exclusive_scan_u32(c, flag, scan, n, tot);
            if (rc) return rc;
            CompactArgs ca;
            std::memset(&ca, 0, sizeof(ca));
            double *arrs[12] = {s->x, s->y, s->z, s->vx, s->vy, s->vz, s->u, s->h,
                                s->ax, s->ay, s->az, s->dudt};
            static const char *tn[12] = {"pt0", "pt1", "pt2", "pt3", "pt4", "pt5",
                                         "pt6", "pt7", "pt8", "pt9", "pt10", "pt11"};
            for (int k = 0; k < 12; ++k) {
                if (!arrs[k]) continue;
                ca.d[ca.nd] = arrs[k];
                ca.dt[ca.nd] = wsa<double>(c, tn[ca.nd], (size_t)n);
                if (!ca.dt[ca.nd]) return fail(c, APR_ERR_HIP, "compaction workspace");
                ca.nd += 1;
            }
            ca.lev = s->level;
            ca.levt = wsa<int8_t>(c, "pt_lev", (size_t)n);
            ca.id = s->id;
            ca.idt = wsa<int64_t>(c, "pt_id", (size_t)n);
            ca.org = origin;
            ca.orgt = origin ? wsa<int64_t>(c, "pt_org", (size_t)n) : nullptr;
            ca.chg = changed;
            ca.chgt = wsa<uint8_t>(c, "pt_chg", (size_t)n);
            if (!ca.levt || !ca.idt || !ca.chgt || (origin && !ca.orgt))
                return fail(c, APR_ERR_HIP, "compaction workspace");
            ca.keep = flag;
            ca.pos = scan;
            ca.n = n;
            int64_t m = n - (int64_t)nm;
            hipLaunchKernelGGL(k_compact_gather, dim3(grid(n)), dim3(256), 0, c->stream, ca);
            hipLaunchKernelGGL(k_compact_back, dim3(grid(m)), dim3(256), 0, c->stream, ca, m);
            APR_LAUNCHED(c);
            n = m;
            s->n = n;
        }
    }
    if (made && n > 0)
        APR_HIP(c, hipMemcpyAsync(made, changed, (size_t)n, hipMemcpyDeviceToDevice, c->stream));
    prof_end(c, tok);
    if (*n_split + *n_merged > 0) {  // the particle set changed: cells are stale
        if (!c->in_bins) c->bins_n = -1;
        c->cells_n = -1;
        c->divv_n = -1;
        c->divv_prev_n = -1;
        c->dens_n = -1;
        c->force_n = -1;
    }
    return APR_OK;
}

}  // namespace apr
