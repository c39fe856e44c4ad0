// Generic gather over the symmetric pair relation r_ab < 2 max(h_a, h_b),
// b != a, r_ab > 0: one workgroup of 4 wavefronts per target cell, candidate
// cells from the tree walk chunk by chunk, LDS staging window by window,
// per-target lists built with 16 lanes per target, pair loops with 4 lanes
// per target.  No atomics on the sums: each target accumulates its own terms
// in a fixed order.
//
// OP supplies (T the pair precision, V = vec4_t<T>):
//   static constexpr int NS;            staged vec4 arrays per particle:
//                                       [0] = (position relative to its cell
//                                       centre, normalised mass), and
//                                       [1].w = 1/h
//   V load(int k, int64_t i) const;     array k of particle i (global)
// The op's own[] and nb[] hold these arrays with the w components of [0] and
// [1] exchanged, [0] = (position, 1/h) and [1].w = the mass, so that the list
// tests read one vector per candidate.
//   struct Acc;                         per-lane partial sums of one target
//   void init(Acc &, const V *own) const;
//   void pair(Acc &, const V *own, T dx, T dy, T dz, T r2, const V *nb) const;
//   const uint8_t *act;                 targets to sum for (null: all)
//   void finish(Acc &, int64_t i, const V *own, bool write) const;
//     finish reduces over the target's 4 lanes (all lanes call it) and, if
//     write, stores the target's results.
//   static constexpr int SK, SC;        a staged component the pair sums never
//                                       read (array SK, component SC = 0..3
//                                       for x..w): it carries the candidate's
//                                       slot for the exact edge test
//   static constexpr bool EXACT;        with EXACT, membership is
//                                       r < 2 max(h_a, h_b) of the FP64
//                                       definition: the pair loop tests
//                                       r^2 / h^2 < 4 for both supports in the
//                                       pair precision and decides pairs
//                                       inside the guard band of either edge
//                                       (kBand) in FP64 on absolute positions;
//                                       without it the pair-precision test
//                                       stands (the adjoint: its terms vanish
//                                       at the edge with their derivatives)
//   int32_t *npair;                     optional (EXACT): pairs per target
//                                       (b != a in the support, r = 0 pairs
//                                       included)
// Staged positions are rounded once from FP64 (stage_pos).
#pragma once

#include "search.hpp"

namespace apr {

template <class T>
__device__ inline void set_comp(vec4_t<T> &v, int c, T x)
{
    if (c == 0) v.x = x;
    else if (c == 1) v.y = x;
    else if (c == 2) v.z = x;
    else v.w = x;
}
template <class T>
__device__ inline T get_comp(const vec4_t<T> &v, int c)
{
    return c == 0 ? v.x : (c == 1 ? v.y : (c == 2 ? v.z : v.w));
}

template <class T, class OP, int STAGE>
__device__ __forceinline__ void gather_cell(const Tree &tr, const OP &op, const CandList &pre,
                                            const int64_t cell, int32_t *status, int st_word)
{
    using V = vec4_t<T>;
    constexpr int NS = OP::NS;
    __shared__ int32_t sA[kCandCap], sB[kCandCap];
    __shared__ V stg[NS][STAGE];
    __shared__ uint16_t sub[kWaves][STAGE];
    __shared__ ListsMeta<T, kTCap> s_lm;  // per-target lists, or candidates' metadata
    uint16_t(*tls)[kTCap] = s_lm.tls;
    const MetaBuf<T> &mb = s_lm.meta;
    __shared__ int s_ncand, s_total, s_more, s_tlen[kCell], s_edge;
    __shared__ Walk s_walk;

    const Geo tg = tr.lev[0][cell];
    const int32_t s0 = tr.cs[cell];
    const int cnt = tr.cs[cell + 1] - s0;
    const int w = wave_id(), lane = lane_id(), j = lane & 3;
    const int t = 16 * w + (lane >> 2);  // this lane's target (4 lanes each)
    // op.act (optional): only those targets get their sums; a cell without
    // one is left at once
    const bool valid = t < cnt && (!op.act || op.act[s0 + t] != 0);
    if (op.act) {
        // block vote through per-wavefront flags (no library reduction buffer)
        __shared__ int s_vote[kWaves];
        const int v = __any(valid) ? 1 : 0;  // every lane votes, then lane 0 stores
        if (lane == 0) s_vote[w] = v;
        __syncthreads();
        int f = 0;
        for (int k = 0; k < kWaves; ++k) f |= s_vote[k];
        if (!f) return;
    }
    uint16_t *mylist = tls[t < kCell ? t : 0];
    const double R = 2.0 * (double)tg.hmax;  // targets' own supports

    V own[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        if (valid) own[k] = op.load(k, s0 + t);
        else { own[k].x = T(0); own[k].y = T(0); own[k].z = T(0); own[k].w = T(0); }
    }
    {
        const T m = own[0].w;
        own[0].w = own[1].w;
        own[1].w = m;
    }
    typename OP::Acc acc;
    op.init(acc, own);
    const bool wave_busy = __any(valid);
    const T ra = valid ? T(2) / own[0].w : T(0);
    // guard bands of r^2/h_a^2 and r^2/h_b^2 about 4: kBand R (mt + 2R) / h^2
    // with R = 2h, i.e. kBand (8 + 2 mt / h)
    const T mt = fabs(own[0].x) + fabs(own[0].y) + fabs(own[0].z);
    const T band_a = kBand<T> * (T(8) + T(2) * mt * own[0].w);
    const T band_b0 = kBand<T> * T(8), band_b1 = kBand<T> * T(2) * mt;
    int npairs = 0;
    if (threadIdx.x == 0) s_edge = 0;  // read after the loop's barriers
    // staged: candidates within max(R, 2 h_b) of the target cell's box
    const T ex = (T)tg.ex, ey = (T)tg.ey, ez = (T)tg.ez;
    const T R2c = (T)(R * R);
    auto cell_reach = [&](T x, T y, T z, T hb) -> bool {
        T d2 = pt_box_d2<T>(x, y, z, T(0), T(0), T(0), ex, ey, ez);
        return (d2 < R2c * kReachSlack<T>) | (d2 * hb * hb < T(4) * kReachSlack<T>);
    };

    bool multiwin = false;  // counted once at the end (no global atomics in the loop)
    // candidates walked ahead of this kernel (same radius), else walk here
    const int pre_n = (pre.ncand && pre.rfac == 2.0 && cell < pre.cap) ? pre.ncand[cell] : -1;
    if (pre_n < 0 && w == 0) walk_init(tr, tg, R, true, &s_walk);
    for (int chunk = 0;; ++chunk) {
        // ---- next chunk of candidate cells
        __syncthreads();  // the previous chunk is no longer read
        if (pre_n >= 0) {
            for (int k = threadIdx.x; k < pre_n; k += kSearchThreads)
                sA[k] = pre.cand[cell * kCandCap + k];
            if (threadIdx.x == 0) {
                s_ncand = pre_n;
                s_more = 0;
            }
        } else if (w == 0) {
            int ncl = walk_next(tr, tg, R, true, &s_walk, sA, kCandCap);
            if (lane == 0) {
                s_ncand = ncl;
                s_more = walk_done(tr, &s_walk) ? 0 : 1;
            }
        }
        __syncthreads();
        const int nc = s_ncand;
        const bool more = s_more != 0;
        load_meta<T>(tr, tg, sA, nc, &s_lm.meta);
        __syncthreads();
        // count the staged candidates, two cells per wavefront at a time (four
        // loads in flight)
        auto near = [&](int ci, int ln) {
            const CandMeta<T> x = mb.m[ci];
            if (ln >= (int)mb.bn[ci]) return false;
            V p = op.load(0, x.b0 + ln);
            T hb = op.load(1, x.b0 + ln).w;
            return cell_reach(p.x + x.sx, p.y + x.sy, p.z + x.sz, hb);
        };
        for (int ci = w; ci < nc; ci += 2 * kWaves) {
            const int c1 = ci + kWaves;
            bool h0 = near(ci, lane);
            bool h1 = c1 < nc && near(c1, lane);
            uint64_t m0 = __ballot(h0), m1 = __ballot(h1);
            if (lane == 0) {
                sB[ci] = __popcll(m0);
                if (c1 < nc) sB[c1] = __popcll(m1);
            }
        }
        __syncthreads();
        if (w == 0) {
            int tot = wave_excl_scan_lds(sB, nc);
            if (lane == 0) s_total = tot;
            if (chunk == 0 && (tot > STAGE || more)) multiwin = true;
        }
        __syncthreads();
        const int total = s_total;
        const int nwin = total > STAGE ? (total + STAGE - 1) / STAGE : 1;

        for (int win = 0; win < nwin && total > 0; ++win) {
            const int w0 = win * STAGE;
            const int nstg = min(STAGE, total - w0);
            if (win > 0) {
                // the previous window and its lists are no longer read; the
                // lists took the metadata's place
                __syncthreads();
                load_meta<T>(tr, tg, sA, nc, &s_lm.meta);
                __syncthreads();
            }
            for (int ci = w; ci < nc; ci += kWaves) {
                int o0 = sB[ci], o1 = ci + 1 < nc ? sB[ci + 1] : total;
                if (o1 <= w0 || o0 >= w0 + STAGE || o1 == o0) continue;
                const CandMeta<T> x = mb.m[ci];
                const int32_t b0 = x.b0, bn = mb.bn[ci];
                bool hit = false;
                V p, v;
                if (lane < bn) {
                    p = op.load(0, b0 + lane);
                    v = op.load(1, b0 + lane);
                    p.x = p.x + x.sx;
                    p.y = p.y + x.sy;
                    p.z = p.z + x.sz;
                    hit = cell_reach(p.x, p.y, p.z, v.w);
                    const T m = p.w;  // staged: [0] = (position, 1/h), [1].w = mass
                    p.w = v.w;
                    v.w = m;
                }
                uint64_t m = __ballot(hit);
                int off = o0 + __popcll(m & lanemask_lt()) - w0;
                if (hit && off >= 0 && off < STAGE) {
                    const int64_t b = (int64_t)b0 + lane;
                    stage_pos<T>(tr, tg, x.wrap, b, p);
                    V e[NS];
                    e[0] = p;
                    e[1] = v;
#pragma unroll
                    for (int k = 2; k < NS; ++k) e[k] = op.load(k, b);
                    set_comp<T>(e[OP::SK], OP::SC, slot_bits(T(0), b));
#pragma unroll
                    for (int k = 0; k < NS; ++k) stg[k][off] = e[k];
                }
            }
            __syncthreads();
            if (!wave_busy) continue;
            build_lists<T, true, kListLanes>(
                nstg, stg[0], sub[w], STAGE, &tls[0][0], kTCap, s_tlen,
                [&](int k) {
                    V q;
                    int tt = 16 * w + k;
                    if (tt < cnt) q = op.load(0, s0 + tt);
                    else { q.x = T(0); q.y = T(0); q.z = T(0); q.w = T(0); }
                    return q;
                },
                [&](int k) { return __shfl(ra, 4 * k, kWave); },
                [&](T d2, T Rs2, const V &p) -> bool {
                    // both tests, no branch: the entry is one vector read
                    return (d2 < Rs2 * kReachSlack<T>) | (d2 * p.w * p.w < T(4) * kReachSlack<T>);
                },
                [&](const V &q, T rk, int e) -> bool {
                    const V p = lds_ld4<T>(&stg[0][e]);
                    T hb = p.w;
                    T dx = q.x - p.x, dy = q.y - p.y, dz = q.z - p.z;
                    T r2 = dx * dx + dy * dy + dz * dz;
                    // with the slack, every pair inside either guard band is listed
                    return (r2 < rk * rk * kReachSlack<T>) |
                           (r2 * hb * hb < T(4) * kReachSlack<T>);
                });
            const int tlen = s_tlen[t < kCell ? t : 0];
            if (!valid) continue;
            const T ha_inv2 = own[0].w * own[0].w;
            const bool ownlist = tlen <= kTCap;
            const int len = ownlist ? tlen : nstg;
            for (int k = j; k < len; k += kLanes) {
                int e = ownlist ? mylist[k] : k;
                V nb[NS];
#pragma unroll
                for (int a = 0; a < NS; ++a) nb[a] = lds_ld4<T>(&stg[a][e]);
                T dx = own[0].x - nb[0].x, dy = own[0].y - nb[0].y, dz = own[0].z - nb[0].z;
                T r2 = dx * dx + dy * dy + dz * dz;
                T hb = nb[0].w;
                const T ta = r2 * ha_inv2, tb = r2 * hb * hb;
                bool in = (ta < T(4)) | (tb < T(4));
                if (OP::EXACT) {
                    const int64_t slot_b = slot_of(get_comp<T>(nb[OP::SK], OP::SC));
                    const int64_t slot_a = (int64_t)s0 + t;
                    if ((fabs(ta - T(4)) <= band_a) |
                        (fabs(tb - T(4)) <= band_b0 + band_b1 * hb)) {
                        // inside a guard band: the FP64 decision (rare)
                        atomicAdd(&s_edge, 1);
                        const double r2e = r2_exact(tr, slot_a, slot_b);
                        in = inside_exact(r2e, tr.ph[slot_a]) | inside_exact(r2e, tr.ph[slot_b]);
                    }
                    npairs += (in & (slot_b != slot_a)) ? 1 : 0;
                }
                if (in & (r2 > T(0))) op.pair(acc, own, dx, dy, dz, r2, nb);
            }
        }
        if (!more) break;
    }
    op.finish(acc, s0 + t, own, valid && j == 0);
    if (OP::EXACT) {
        npairs = sum4(npairs);
        if (op.npair && valid && j == 0) op.npair[s0 + t] = npairs;
    }
    __syncthreads();  // s_edge complete
    if (threadIdx.x == 0) {
        if (multiwin && st_word >= 0) atomicAdd(&status[st_word], 1);
        if (s_edge) atomicAdd(&status[ST_EDGE], s_edge);
    }
}

// One workgroup per target cell, cells [0, grid) with the grid from the
// host's estimate of the cell count; the REST launch strides over any cells
// from `first` on, nearly always none (a loop around the search body costs it
// registers, hence two kernels).
template <class T, class OP, int STAGE, bool REST>
__device__ void gather_pairs(const Tree &tr, const OP &op, const CandList &pre, int32_t *status,
                             int st_word, int64_t first)
{
    const int64_t nc = tr.hdr->ncells;
    if (!REST) {
        const int64_t cell = first_cell(blockIdx.x, gridDim.x, nc);
        if (cell >= 0) gather_cell<T, OP, STAGE>(tr, op, pre, cell, status, st_word);
        return;
    }
    for (int64_t cell = first + blockIdx.x; cell < nc; cell += gridDim.x) {
        gather_cell<T, OP, STAGE>(tr, op, pre, cell, status, st_word);
        __syncthreads();  // the next cell reuses the LDS
    }
}

}  // namespace apr
