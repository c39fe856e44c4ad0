// Density and smoothing length: the h-rho Newton iteration of every particle
// (the paper defers to Phantom's iterative solve, Sec. 2.2):
//   rho_a = sum_b m_b W(r_ab, h_a)  (b = a included),  h_a = hfact (m_a/rho_a)^(1/3),
//   F(h) = rho_sum(h) - m_a (hfact/h)^3,  F'(h) = sum_b m_b dW/dh + 3 m_a hfact^3/h^4,
//   Omega_a = 1 + h_a/(3 rho_a) sum_b m_b dW_ab/dh_a.
// The update is Newton's with Halley's correction from F'' (cubic
// convergence: one pass fewer for guesses off by about 1e-3):
//   F'' = sum_b m_b d2W/dh2 - 12 m_a hfact^3/h^5,
//   d2W/dh2 = (12 f + 8 q f' + q^2 f'')/(pi h^5),
//   h <- h - (F/F') / (1 - F F''/(2 F'^2))   (plain Newton if |F F''/(2 F'^2)| >= 1/2).
// It stops when |dh| < tol h; the h reported is the one the last sums were
// taken at.  A Halley step with |dh| < sqrt(tol) h also ends it: its
// remaining error is of order (dh/h)^3 h, far below tol h, so h + dh is
// reported without another pass, with rho and the h-derivative sum of Omega
// carried to it by their Taylor series (rho to second order, errors of order
// (dh/h)^3 and (dh/h)^2 <= tol).  The neighbour count reported is the one at
// h + dh: the pass's own when no pair it evaluated lies between the two
// supports and it evaluated every candidate within 2 (h + dh); else one
// taken again over the target's list, if that list covers the new support;
// else the step waits for another pass.  If F' <= 0 the step is
// h_fact (m/rho_sum)^(1/3); every step is clamped to [h/2, 2h].
//
// Membership r_ab < 2 h_a is tested in the pair precision and, inside a
// guard band about the edge, decided again in FP64 on absolute positions
// (exactly the neighbour export's predicate), so the pairs summed and the
// count reported are those of the FP64 definition in both forms.
//
// Kernel (M4 or Wendland C2, support 2h, a template parameter): W = f(q)/(pi h^3),
// q = r/h, so dW/dh = -(3f + q f')/(pi h^4).  Sums carry the normalised mass
// 2^-level; m0/pi is applied once in FP64.
//
// Pair arithmetic in T (float: cell-relative coordinates, Kahan-compensated
// sums; double: the same code in FP64).  The Newton update and its
// convergence test are FP64 in both forms.
//
// One workgroup (4 wavefronts) per target cell of up to 64 particles; a
// wavefront takes 16 targets.  The candidates within reach of some
// wavefront's targets are staged in LDS; each wavefront then lists, per
// target, the staged entries within 2 sigma h (4 targets at a time, 16 lanes
// each), and every Newton pass sums a target's list with 4 lanes.  If a
// target's 2h outgrows the staged radius the workgroup searches and stages
// again with the larger radius (bounded: h at most doubles per Newton step,
// max_iter).
#include "search.hpp"
#include "sph_kernel.hpp"

namespace apr {

namespace {

constexpr float kSigma = 1.01f;  // staged radius margin over 2 h_max

template <class T>
struct StageCap;
template <>
struct StageCap<float> {
    static constexpr int value = 1024;
};
template <>
struct StageCap<double> {
    static constexpr int value = 768;
};
// Per-target list capacity (density).  A uniform medium has about 57
// neighbours within 2h, but at an interface of masses differing eightfold
// (the shock box) half a heavy particle's neighbours are light, its h grows
// by about a fifth and its count reaches about 100; a longer list would
// leave the target walking the whole staged set every pass.
constexpr int kDTCap = 128;

template <class T>
struct DensArgs {
    Tree tree;
    const vec4_t<T> *pm;  // position relative to own cell centre, normalised mass
    double *h;            // in: guess, out: converged
    T *rho;
    T *omega;
    int32_t *nneigh;
    int32_t *iters;
    T *dnn;
    float *hmax_new;      // per cell
    CandList pre;         // candidate cells walked ahead (radius 2 sigma hmax)
    double m0, hfact, tol;
    double m0_pi, hfact3; // m0 / pi and hfact^3, computed once on the host (kept in
                          // scalar registers, not in vector registers across the kernel)
    double tol_take;      // sqrt(tol): a Halley step below it ends the iteration
    double hlim;          // periodic boxes: h must stay below this (0: no limit)
    int max_iter;
    int32_t *status;
    const uint8_t *active;  // targets to solve (null: all); the others keep h, rho, Omega
};

// A staged density candidate carries its mass 2^-level (an exact power of
// two, zero mantissa) with a tag in the low 14 mantissa bits: its candidate
// cell's index in the chunk (8 bits) and its lane in that cell (6 bits).
// The slot is then cs[sA[ci]] + lane, needed only by the FP64 edge test.
constexpr uint32_t kTagBits = 14;
__device__ inline float tag_mass(float m, int ci, int lane)
{
    return __int_as_float(__float_as_int(m) | (ci << 6) | lane);
}
__device__ inline double tag_mass(double m, int ci, int lane)
{
    return __longlong_as_double(__double_as_longlong(m) | (long long)((ci << 6) | lane));
}
__device__ inline float untag_mass(float w)
{
    return __int_as_float(__float_as_int(w) & ~((1 << kTagBits) - 1));
}
__device__ inline double untag_mass(double w)
{
    return __longlong_as_double(__double_as_longlong(w) & ~((1ll << kTagBits) - 1));
}
__device__ inline int tag_of(float w) { return __float_as_int(w) & ((1 << kTagBits) - 1); }
__device__ inline int tag_of(double w)
{
    return (int)(__double_as_longlong(w) & ((1ll << kTagBits) - 1));
}

// Per-lane partial sums of one Newton evaluation (kernel K).
template <class T, int K>
struct DSum {
    Acc<T> w, d;  // sum m f, sum m (3f + q f'), compensated
    T k;          // sum m (12 f + 8 q f' + q^2 f''): only Halley's correction of the
                  // Newton step uses it, so a plain sum suffices (one register fewer)
    int cnt;       // neighbours in the low 16 bits, those at r = 0 above
    T dmin;
    T emin;        // min |r^2 - R2hi| over every pair evaluated, in or out
    __device__ void zero()
    {
        w.zero();
        d.zero();
        k = T(0);
        cnt = 0;
        dmin = T(3.0e38);
        emin = T(3.0e38);
    }
    // wt: the staged mass with its candidate tag; inside the guard band
    // R2lo <= r^2 <= R2hi (R^2 -+ band) edge(wt) decides membership in FP64,
    // below it the pair is in, above it out
    template <class Edge>
    __device__ void pair(T dx, T dy, T dz, T wt, T R2lo, T R2hi, T hinv, Edge edge)
    {
        T r2 = dx * dx + dy * dy + dz * dz;
        const T e = fabs(r2 - R2hi);
        emin = emin < e ? emin : e;
        bool in = r2 < R2lo;
        if (!in && r2 <= R2hi) in = edge(wt);
        if (in) {
            const T m = untag_mass(wt);
            T r = psqrt(r2);
            const T q = r * hinv;
            T f, df, d2f;
            Kern<K>::template eval<T, 2>(q, f, df, d2f);
            const T g = T(3) * f + q * df;
            const T kk = T(12) * f + q * (T(8) * df + q * d2f);
            w.add(m * f);
            d.add(m * g);
            k += m * kk;
            bool zero = !(r2 > T(0));
            cnt += zero ? 0x10001 : 1;
            T rr = zero ? T(3.0e38) : r;
            dmin = dmin < rr ? dmin : rr;
        }
    }
};

// Candidate particle `lane` of candidate cell ci in the target cell's frame;
// false for lanes beyond the cell's size or out of every wavefront's reach.
template <class T>
__device__ inline bool cand_point(const vec4_t<T> *pm, const MetaBuf<T> &mb, int ci, int lane,
                                  const WaveBoxes<T> &B, vec4_t<T> &p)
{
    const CandMeta<T> x = mb.m[ci];
    if (lane >= (int)mb.bn[ci]) return false;
    p = pm[x.b0 + lane];
    p.x = p.x + x.sx;
    p.y = p.y + x.sy;
    p.z = p.z + x.sz;
    return wave_reach<T, false>(B, p.x, p.y, p.z, T(0));
}

// Counts, per candidate cell, the particles within reach of some
// wavefront's targets (into sB), and keeps which lanes they are (smask).
// Two cells per wavefront at a time, so that two loads are in flight.
template <class T>
__device__ inline void count_cands(const vec4_t<T> *pm, const MetaBuf<T> &mb, int nc,
                                   const WaveBoxes<T> &B, int32_t *sB, uint64_t *smask)
{
    const int w = wave_id(), lane = lane_id();
    for (int ci = w; ci < nc; ci += 2 * kWaves) {
        const int c1 = ci + kWaves;
        vec4_t<T> p0, p1;
        bool h0 = cand_point<T>(pm, mb, ci, lane, B, p0);
        bool h1 = c1 < nc && cand_point<T>(pm, mb, c1, lane, B, p1);
        uint64_t m0 = __ballot(h0), m1 = __ballot(h1);
        if (lane == 0) {
            sB[ci] = __popcll(m0);
            smask[ci] = m0;
            if (c1 < nc) {
                sB[c1] = __popcll(m1);
                smask[c1] = m1;
            }
        }
    }
}

// Stages everything counted when it fits one window: the lanes counting
// found (smask) at the offsets of the scan (sB), without testing the reach
// again.
template <class T>
__device__ inline void stage_counted(const Tree &tr, const Geo &tg, const vec4_t<T> *pm,
                                     const MetaBuf<T> &mb, const int32_t *sB,
                                     const uint64_t *smask, int nc, vec4_t<T> *stg)
{
    const int w = wave_id(), lane = lane_id();
    for (int ci = w; ci < nc; ci += kWaves) {
        const uint64_t m = smask[ci];
        if (!((m >> lane) & 1ull)) continue;
        const int off = sB[ci] + __popcll(m & lanemask_lt());
        const int64_t b = (int64_t)mb.m[ci].b0 + lane;
        vec4_t<T> p;
        p.w = pm[b].w;
        stage_pos<T>(tr, tg, mb.m[ci].wrap, b, p);
        p.w = tag_mass(p.w, ci, lane);
        stg[off] = p;
    }
}

// Stages the counted candidates with staged offset in [w0, w0 + STAGE):
// positions in the target cell's frame.  sB holds each candidate cell's
// first offset.
// The staged entry: position rounded once from FP64 (stage_pos), the mass
// tagged with (ci, lane).  The reach test is cand_point's, as in counting, so
// that the staged set is exactly the counted one.
template <class T, int STAGE>
__device__ inline void stage_window(const Tree &tr, const Geo &tg, const vec4_t<T> *pm,
                                    const MetaBuf<T> &mb, const int32_t *sB, int nc, int total,
                                    const WaveBoxes<T> &B, int w0, vec4_t<T> *stg)
{
    const int w = wave_id(), lane = lane_id();
    for (int ci = w; ci < nc; ci += kWaves) {
        int o0 = sB[ci], o1 = ci + 1 < nc ? sB[ci + 1] : total;
        if (o1 <= w0 || o0 >= w0 + STAGE || o1 == o0) continue;
        vec4_t<T> p;
        bool hit = cand_point<T>(pm, mb, ci, lane, B, p);
        uint64_t m = __ballot(hit);
        int off = o0 + __popcll(m & lanemask_lt()) - w0;
        if (hit && off >= 0 && off < STAGE) {
            stage_pos<T>(tr, tg, mb.m[ci].wrap, (int64_t)mb.m[ci].b0 + lane, p);
            p.w = tag_mass(p.w, ci, lane);
            stg[off] = p;
        }
    }
}

// ACT: only the targets a.active flags are solved (individual timesteps); a
// separate instantiation, so that the full pass carries none of it.
template <class T, int K, bool ACT>
__device__ __forceinline__ void density_cell(const DensArgs<T> &a, const int64_t cell)
{
    using V = vec4_t<T>;
    constexpr int STAGE = StageCap<T>::value;
    __shared__ int32_t sA[kCandCap], sB[kCandCap];
    __shared__ V stg[STAGE];
    __shared__ ListsMeta<T, kDTCap> s_lm;  // per-target lists, or candidates' metadata
    uint16_t(*tls)[kDTCap] = s_lm.tls;
    // the list builders' scratch; between counting and staging, which lanes
    // of each candidate cell were counted
    __shared__ __attribute__((aligned(16))) uint16_t sub[kWaves][kSubCap];
    static_assert(sizeof(sub) >= kCandCap * sizeof(uint64_t), "counted-lane masks");
    uint64_t *smask = reinterpret_cast<uint64_t *>(&sub[0][0]);
    __shared__ int s_ncand, s_total, s_flag[kWaves], s_tlen[kCell];
    __shared__ double s_red[kWaves];
    __shared__ int s_more, s_edge;
    __shared__ Walk s_walk;
    __shared__ WaveBoxes<T> s_wb;
    __shared__ double s_Rw[kWaves];  // each wavefront's staged reach
    // each target's results until the final store (registers are scarce)
    struct Out {
        T rho, om, dnn;
        int nn;  // neighbour count; negative: the solve hit max_iter
    };
    __shared__ Out s_out[kCell];

    const Tree &tr = a.tree;
    const Geo tg = tr.lev[0][cell];
    const int32_t s0 = tr.cs[cell];
    const int cnt = tr.cs[cell + 1] - s0;
    const int w = wave_id(), lane = lane_id(), j = lane & 3;
    const int t = 16 * w + (lane >> 2);   // this lane's target (4 lanes each)
    const bool mine = t < cnt;
    const bool valid = mine && (!ACT || a.active[s0 + t] != 0);
    bool any_valid = true;
    if (ACT) {
        // block vote through the wavefront flags (no library reduction buffer)
        const int v = __any(valid) ? 1 : 0;
        if (lane == 0) s_flag[w] = v;
        __syncthreads();
        int f = 0;
        for (int k = 0; k < kWaves; ++k) f |= s_flag[k];
        any_valid = f != 0;
        __syncthreads();  // s_flag is written again below
    }
    if (!any_valid) {
        // nothing to solve here: the cell's h_max from the stored h
        double m = wave_max64(mine ? a.h[s0 + t] : 0.0);
        if (lane_id() == 0) s_red[wave_id()] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            double hm = 0.0;
            for (int k = 0; k < kWaves; ++k) hm = fmax(hm, s_red[k]);
            a.hmax_new[cell] = f_up(hm);
        }
        return;
    }

    double h = valid ? a.h[s0 + t] : 0.0;
    // per target, in LDS (registers are scarce): the reach of its list (2
    // sigma h), the list's length and the Newton passes taken
    __shared__ float s_Rt[kCell];
    __shared__ uint16_t s_itc[kCell];  // max_iter <= 1000
    // results are kept in s_out and stored once after the iteration (no global
    // writes inside the loop: every barrier waits for outstanding ones)
    // work counters of the block (thread 0), added once at the end
    // (in LDS, thread 0's: registers are scarce)
    __shared__ int c_restage, c_direct, c_windows, c_passes;
    bool done = !valid;
    bool recount = false;  // took an accepted step that counts again at the new h
    V tp;
    if (valid) tp = a.pm[s0 + t];
    else { tp.x = T(0); tp.y = T(0); tp.z = T(0); tp.w = T(0); }
    uint16_t *mylist = tls[t < kCell ? t : 0];
    // FP64 decision for a pair inside the guard band: the candidate's slot
    // from its tag and the chunk's candidate cells, then the exact predicate
    // at this lane's current h (rare: a few pairs per thousand targets)
    auto edge = [&](T wt, double hx) -> bool {
        const int tag = tag_of(wt);
        const int64_t b = (int64_t)tr.cs[sA[tag >> 6]] + (tag & 63);
        atomicAdd(&s_edge, 1);
        return inside_exact(r2_exact(tr, s0 + t, b), hx);
    };

    // staged reach of each wavefront's targets (2 sigma of its largest h) and
    // of the whole cell (the tree walk's radius)
    double R;
    {
        wave_box<T>(&s_wb, valid, tp.x, tp.y, tp.z);
        double m = wave_max64(h);
        if (lane == 0) s_red[w] = m;
        __syncthreads();
        R = 0.0;
        for (int k = 0; k < kWaves; ++k) R = fmax(R, 2.0 * (double)kSigma * s_red[k]);
        if (threadIdx.x == 0) {
            for (int k = 0; k < kWaves; ++k) {
                double rw = 2.0 * (double)kSigma * s_red[k];
                s_Rw[k] = rw;
                s_wb.R2[k] = 16 * k < cnt ? (T)(rw * rw) : T(-1);
            }
            s_edge = 0;
            c_restage = c_direct = c_windows = c_passes = 0;
        }
        if (threadIdx.x < kCell) {
            s_Rt[threadIdx.x] = 0.0f;
            s_itc[threadIdx.x] = 0;
            s_tlen[threadIdx.x] = 0;
        }
    }

    // Every new search follows a Newton step that grew some h, and every
    // pass is a Newton step for each pending target: max_iter bounds both.
    // A cell whose candidates span several chunks of the tree walk walks
    // again in every pass (multi); otherwise the candidates of the last walk
    // stay, and with a single window the staged set and the lists too.
    bool search = true;
    bool multi = false;
    bool lists = false;    // per-target lists valid (single chunk and window only)
    int nc = 0, total = 0, nwin = 1;
    for (int pass = 0; pass <= a.max_iter; ++pass) {
        DSum<T, K> S;
        S.zero();
        const bool wave_busy = __any(!done);
        const bool walking = search || multi;
        // the first search can take the candidates walked ahead of this kernel
        int pre_n = -1;
        if (pass == 0 && a.pre.ncand && cell < a.pre.cap && R <= a.pre.rfac * (double)tg.hmax)
            pre_n = a.pre.ncand[cell];
        const bool use_pre = walking && pre_n >= 0;
        if (walking && !use_pre) {
            __syncthreads();
            if (w == 0) walk_init(tr, tg, R, false, &s_walk);
            if (search && pass > 0 && threadIdx.x == 0) c_restage += 1;
        }
        for (int chunk = 0;; ++chunk) {
            bool last = true;
            if (walking) {
                // ---- next chunk of candidate cells, staged counts and offsets
                __syncthreads();
                if (use_pre) {
                    for (int k = threadIdx.x; k < pre_n; k += kSearchThreads)
                        sA[k] = a.pre.cand[cell * kCandCap + k];
                    if (threadIdx.x == 0) {
                        s_ncand = pre_n;
                        s_more = 0;
                    }
                } else if (w == 0) {
                    int ncl = walk_next(tr, tg, R, false, &s_walk, sA, kCandCap);
                    if (lane == 0) {
                        s_ncand = ncl;
                        s_more = walk_done(tr, &s_walk) ? 0 : 1;
                    }
                }
                __syncthreads();
                nc = s_ncand;
                last = s_more == 0;
                if (!last) multi = true;
                load_meta<T>(tr, tg, sA, nc, &s_lm.meta);
                __syncthreads();
                count_cands<T>(a.pm, s_lm.meta, nc, s_wb, sB, smask);
                __syncthreads();
                if (w == 0) {
                    int tot = wave_excl_scan_lds(sB, nc);
                    if (lane == 0) {
                        s_total = tot;
                        if (pass == 0 && chunk == 0 && (tot > STAGE || !last)) c_direct = 1;
                    }
                }
                __syncthreads();
                total = s_total;
                nwin = total > STAGE ? (total + STAGE - 1) / STAGE : 1;
                lists = false;
                if (nwin == 1) {
                    stage_counted<T>(tr, tg, a.pm, s_lm.meta, sB, smask, nc, stg);
                    __syncthreads();
                }
            }
            // ---- this chunk's part of one Newton evaluation, window by window
            for (int win = 0; win < nwin && total > 0; ++win) {
                int w0 = win * STAGE;
                int nstg = min(STAGE, total - w0);
                if (nwin > 1) {
                    // the previous window and its lists are no longer read; the
                    // lists took the metadata's place
                    __syncthreads();
                    load_meta<T>(tr, tg, sA, nc, &s_lm.meta);
                    __syncthreads();
                    stage_window<T, STAGE>(tr, tg, a.pm, s_lm.meta, sB, nc, total, s_wb, w0, stg);
                    __syncthreads();
                }
                if (!wave_busy) continue;
                if (!lists) {
                    // this target's candidates within 2 sigma h (with margin)
                    if (j == 0) s_Rt[t] = done ? 0.0f : (float)(2.0 * (double)kSigma * h);
                    wave_sync();
                    build_lists<T, false, kListLanes>(
                        nstg, stg, sub[w], kSubCap, &tls[0][0], kDTCap, s_tlen,
                        [&](int k) {
                            V q;
                            int tt = 16 * w + k;
                            if (tt < cnt) q = a.pm[s0 + tt];
                            else { q.x = T(0); q.y = T(0); q.z = T(0); q.w = T(0); }
                            return q;
                        },
                        [&](int k) { return (T)s_Rt[16 * w + k]; },
                        [&](T d2, T Rs2, const V &) { return d2 < Rs2; },
                        [&](const V &q, T rk, int e) {
                            V p = stg[e];
                            T dx = q.x - p.x, dy = q.y - p.y, dz = q.z - p.z;
                            return dx * dx + dy * dy + dz * dz < rk * rk;
                        });
                }
                if (done) continue;
                const int tlen = s_tlen[t];
                T hf = (T)h;
                T hinv = T(1) / hf;
                T R2 = T(4) * hf * hf;
                const T band = edge_band<T>(tp, T(2) * hf);
                const T R2lo = R2 - band, R2hi = R2 + band;
                const double hx = (double)hf;  // the h these sums are reported at
                auto ed = [&](T wt) { return edge(wt, hx); };
                if (tlen <= kDTCap) {
                    // two entries per step (same order per lane), both reads in flight
                    int k = j;
                    for (; k + kLanes < tlen; k += 2 * kLanes) {
                        const int e0 = mylist[k], e1 = mylist[k + kLanes];
                        const V p0 = lds_ld4<T>(&stg[e0]), p1 = lds_ld4<T>(&stg[e1]);
                        S.pair(tp.x - p0.x, tp.y - p0.y, tp.z - p0.z, p0.w, R2lo, R2hi, hinv, ed);
                        S.pair(tp.x - p1.x, tp.y - p1.y, tp.z - p1.z, p1.w, R2lo, R2hi, hinv, ed);
                    }
                    if (k < tlen) {
                        const V p = lds_ld4<T>(&stg[mylist[k]]);
                        S.pair(tp.x - p.x, tp.y - p.y, tp.z - p.z, p.w, R2lo, R2hi, hinv, ed);
                    }
                } else {
                    // own list overflowed: walk the whole window
                    for (int k = j; k < nstg; k += kLanes) {
                        V p = stg[k];
                        S.pair(tp.x - p.x, tp.y - p.y, tp.z - p.z, p.w, R2lo, R2hi, hinv, ed);
                    }
                }
            }
            if (threadIdx.x == 0) c_windows += nwin;
            if (last) break;
        }
        search = false;
        lists = !multi && nwin == 1;
        if (threadIdx.x == 0) c_passes += 1;
        // ---- FP64 Newton step of this lane's target (its 4 lanes agree)
        double needR = 0.0;
        bool pending = false;
        S.w.template reduce<kLanes>();
        S.d.template reduce<kLanes>();
        S.k = sum4(S.k);
        int cnt4 = sum4(S.cnt);
        int nn = cnt4 & 0xffff, nzero = cnt4 >> 16;
        T dmin = min4(S.dmin);
        const T emin = min4(S.emin);
        if (!done) {
            const double W = S.w.value(), D = S.d.value();
            const double hh = (double)(T)h;
            const double hi = 1.0 / hh, c0 = a.m0_pi * hi * hi * hi;
            const double ma = a.m0 * (double)tp.w;
            const double rhos = c0 * W;                      // rho_sum(hh)
            const double drho = -c0 * hi * D;                // d rho_sum / dh
            const double d2rho = c0 * hi * hi * (double)S.k; // d2 rho_sum / dh2
            const double rhoh = ma * a.hfact3 * hi * hi * hi;
            const double F = rhos - rhoh, dF = drho + 3.0 * rhoh * hi;
            double hn;
            bool halley = false;
            if (dF > 0.0) {
                const double d2F = d2rho - 12.0 * rhoh * hi * hi;
                const double x = F * d2F / (2.0 * dF * dF);
                halley = fabs(x) < 0.5;
                hn = hh - F / (halley ? dF * (1.0 - x) : dF);
            } else {
                hn = a.hfact * cbrt(ma / rhos);
            }
            hn = fmin(fmax(hn, 0.5 * hh), 2.0 * hh);
            const double dh = hn - hh;
            bool conv = fabs(dh) < a.tol * hh;
            // An accepted step reports hn with the neighbour count at hn.  That
            // count is this pass's when every candidate within 2 hn was
            // evaluated (the target's list reach and the staged reach cover it)
            // and no evaluated pair lies between the supports at hh and hn: a
            // pair there has |r^2 - R^2| in the pair precision within
            // |4 hn^2 - 4 hh^2| plus the rounding of r^2 (below a quarter of
            // the guard band) and of R^2, so |r^2 - R2hi| within that plus
            // the band.  Otherwise the target's own list, if valid for
            // another pass and holding the new support, counts again.
            const bool small = !conv && halley && fabs(dh) < a.tol_take * hh;
            const double hcov = 2.0 * hn * (1.0 + 1.0 / 1024);
            const double Rt = (double)s_Rt[t];
            const int tlen = s_tlen[t];
            const bool covered = hcov < fmin(Rt, s_Rw[w]);
            const double shell = fabs(4.0 * (hn * hn - hh * hh)) +
                                 2.0 * (double)edge_band<T>(tp, T(2) * (T)hh) +
                                 0x1p-20 * (4.0 * hh * hh);
            const bool same = covered && (double)emin > shell;
            const bool relist = lists && tlen <= kDTCap && hcov < Rt;
            const bool take = small && (same || relist);
            conv = conv || take;
            const int itc = s_itc[t] + 1;
            if (j == 0) s_itc[t] = (uint16_t)itc;
            if (conv || itc >= a.max_iter) {
                done = true;
                recount = take && !same;
                h = take ? hn : hh;
                if (j == 0) {
                    // The accepted step carries rho (second order) and Omega =
                    // 1 + h rho'/(3 rho) (first order) from hh to hh + dh
                    const double om = 1.0 - D / (3.0 * W);
                    Out o;
                    o.rho = (T)(take ? rhos + dh * (drho + 0.5 * dh * d2rho) : rhos);
                    o.om = (T)(take ? om + (dh / 3.0) * (drho + hh * (d2rho - drho * drho / rhos)) /
                                               rhos
                                    : om);
                    o.dnn = nzero >= 2 ? T(0)
                                       : (dmin >= T(3.0e38) ? T(__builtin_huge_val()) : dmin);
                    o.nn = conv ? nn : -1 - nn;
                    s_out[t] = o;
                }
            } else {
                h = hn;
                pending = true;
                if (2.0 * hn > Rt) lists = false;   // own list too short now
                if (2.0 * hn > s_Rw[w]) needR = 2.0 * (double)kSigma * hn;
            }
        }
        // ---- a target that took its last step counts its neighbours again at
        // the new h, over its own list (still staged: nothing is restaged
        // before the block-wide step below)
        if (__any(recount)) {
            const T hf = (T)h;
            const T R2 = T(4) * hf * hf;
            const T band = edge_band<T>(tp, T(2) * hf);
            const int len = recount ? s_tlen[t] : 0;
            int c = 0;
            for (int k = j; k < len; k += kLanes) {
                const V p = lds_ld4<T>(&stg[mylist[k]]);
                const T dx = tp.x - p.x, dy = tp.y - p.y, dz = tp.z - p.z;
                const T r2 = dx * dx + dy * dy + dz * dz;
                bool in = r2 < R2;
                if (fabs(r2 - R2) <= band) in = edge(p.w, h);
                c += in ? 1 : 0;
            }
            c = sum4(c);
            if (recount && j == 0) s_out[t].nn = c;
            recount = false;
        }
        // ---- block-wide: anything pending?  a larger search radius needed?
        {
            double m = wave_max64(needR);
            int pw = __any(pending) ? 1 : 0;
            int lw = __any(!lists) ? 1 : 0;
            __syncthreads();
            if (lane == 0) {
                s_red[w] = m;
                s_flag[w] = pw | (lw << 1);
            }
            __syncthreads();
            double need = 0.0;
            int fl = 0;
            for (int k = 0; k < kWaves; ++k) {
                need = fmax(need, s_red[k]);
                fl |= s_flag[k];
            }
            if (!(fl & 1)) break;
            if (fl & 2) lists = false;
            if (need > 0.0) {
                // a wavefront's reach no longer covers some 2h: widen it
                for (int k = 0; k < kWaves; ++k) {
                    double rw = s_red[k] > 0.0 ? fmax(s_red[k], 1.25 * s_Rw[k]) : s_Rw[k];
                    R = fmax(R, rw);
                }
                __syncthreads();  // every thread has read s_red and the old reach
                if (threadIdx.x == 0)
                    for (int k = 0; k < kWaves; ++k) {
                        double rw = s_red[k] > 0.0 ? fmax(s_red[k], 1.25 * s_Rw[k]) : s_Rw[k];
                        s_Rw[k] = rw;
                        if (16 * k < cnt) s_wb.R2[k] = (T)(rw * rw);
                    }
                search = true;
            }
        }
    }

    // ---- results and counters
    if (valid && j == 0) {
        int64_t i = s0 + t;
        Out o = s_out[t];
        a.h[i] = h;
        a.rho[i] = o.rho;
        a.omega[i] = o.om;
        if (a.nneigh) a.nneigh[i] = o.nn >= 0 ? o.nn : -1 - o.nn;
        if (a.iters) a.iters[i] = s_itc[t];
        if (a.dnn) a.dnn[i] = o.dnn;
        if (o.nn < 0) atomicAdd(&a.status[ST_NOCONV], 1);
        if (a.hlim > 0.0 && !(h < a.hlim)) atomicOr(&a.status[ST_RANGE], 1);
        // the staging slack covers the guard band while |t|_1 < 126 R
        if ((double)(fabs(tp.x) + fabs(tp.y) + fabs(tp.z)) >= 252.0 * h)
            atomicAdd(&a.status[ST_BAND], 1);
    }
    __syncthreads();  // s_edge complete
    if (threadIdx.x == 0) {
        if (s_edge) atomicAdd(&a.status[ST_EDGE], s_edge);
        if (c_restage) atomicAdd(&a.status[ST_RESTAGE], c_restage);
        if (c_direct) atomicAdd(&a.status[ST_DENS_DIRECT], c_direct);
        atomicAdd(&a.status[ST_WINDOWS], c_windows);
        atomicAdd(&a.status[ST_PASSES], c_passes);
    }
    // ---- new h_max of the cell for the force search
    {
        double m = wave_max64(valid ? h : (ACT && t < cnt ? a.h[s0 + t] : 0.0));
        __syncthreads();
        if (lane == 0) s_red[w] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            double hm = 0.0;
            for (int k = 0; k < kWaves; ++k) hm = fmax(hm, s_red[k]);
            a.hmax_new[cell] = f_up(hm);
        }
    }
}

// One workgroup per target cell, cells [0, grid) with the grid from the
// host's estimate of the cell count; a second launch (REST) strides over any
// cells from `first` on, nearly always none.  Two kernels rather than one
// loop: a loop around the search body costs it registers.
template <class T, int K, bool REST, bool ACT>
__global__ __launch_bounds__(kSearchThreads, kBlocksPerCU<T>) void k_density(DensArgs<T> a,
                                                                              int64_t first)
{
    const int64_t nc = a.tree.hdr->ncells;
    if (!REST) {
        const int64_t cell = first_cell(blockIdx.x, gridDim.x, nc);
        if (cell >= 0) density_cell<T, K, ACT>(a, cell);
        return;
    }
    for (int64_t cell = first + blockIdx.x; cell < nc; cell += gridDim.x) {
        density_cell<T, K, ACT>(a, cell);
        __syncthreads();  // the next cell reuses the LDS
    }
}

template <class T, int K, bool ACT>
void launch_density_a(apr_ctx *c, const DensArgs<T> &a, int64_t grid, int tok)
{
    hipLaunchKernelGGL((k_density<T, K, false, ACT>), dim3((unsigned)grid), dim3(kSearchThreads),
                       0, c->stream, a, (int64_t)0);
    prof_end(c, tok);  // the timed pass: the REST launch is nearly always empty
    hipLaunchKernelGGL((k_density<T, K, true, ACT>), dim3(kRestGrid), dim3(kSearchThreads), 0,
                       c->stream, a, grid);
}

template <class T, int K>
void launch_density_k(apr_ctx *c, const DensArgs<T> &a, int64_t grid, int tok)
{
    if (a.active) launch_density_a<T, K, true>(c, a, grid, tok);
    else launch_density_a<T, K, false>(c, a, grid, tok);
}

template <class T>
void launch_density(apr_ctx *c, const DensArgs<T> &a, int64_t grid, int tok)
{
    if (c->p.kernel == APR_KERNEL_WC2) launch_density_k<T, kWC2>(c, a, grid, tok);
    else launch_density_k<T, kM4>(c, a, grid, tok);
}

}  // namespace

Tree make_tree(apr_ctx *c, const apr_state *s)
{
    Tree t;
    t.hdr = cell_hdr(c);
    t.cs = cell_start(c);
    for (int k = 0; k <= kMaxLev; ++k) t.lev[k] = k <= c->nlev ? cell_level(c, k) : nullptr;
    t.nlev = c->nlev;
    t.box = make_box(c->p);
    t.px = s->x;
    t.py = s->y;
    t.pz = s->z;
    t.ph = s->h;
    return t;
}

int density(apr_ctx *c, apr_state *s, void *rho, void *omega, int32_t *nneigh, int32_t *iters,
            const uint8_t *active)
{
    if (c->cells_n != s->n) return fail(c, APR_ERR_INVALID, "apr_build_cells first");
    if (!rho || !omega) return fail(c, APR_ERR_INVALID, "rho and omega are required");
    const int64_t grid = c->node_grid[0];
    float *hmax_new = wsa<float>(c, "hmax_new", (size_t)c->node_cap[0]);
    int32_t *st = c->d_status;
    Tree tr = make_tree(c, s);
    // periodic: 2 h < box / 4 on every axis
    double hlim = 0.0;
    if (c->p.periodic) {
        hlim = 1e300;
        for (int k = 0; k < 3; ++k) hlim = fmin(hlim, 0.125 * (c->p.box_hi[k] - c->p.box_lo[k]));
    }
    CandList pre;
    int rc0 = cand_pre(c, tr, false, 2.0 * (double)kSigma, &pre, active);
    if (rc0) return rc0;
    int tok = prof_begin(c, APR_PROF_DENSITY);
    if (c->p.precision == APR_FP32) {
        DensArgs<float> a;
        a.tree = tr;
        a.pm = wsa<float4>(c, "pm32", (size_t)s->n);
        a.h = s->h;
        a.rho = (float *)rho;
        a.omega = (float *)omega;
        a.nneigh = nneigh;
        a.iters = iters;
        a.dnn = wsa<float>(c, "dnn32", (size_t)s->capacity);
        a.hmax_new = hmax_new;
        a.pre = pre;
        a.m0 = c->p.m0;
        a.hfact = c->p.hfact;
        a.m0_pi = c->p.m0 / kPi;
        a.hfact3 = c->p.hfact * c->p.hfact * c->p.hfact;
        a.tol = c->p.tol_h;
        a.tol_take = std::sqrt(c->p.tol_h);
        a.hlim = hlim;
        a.max_iter = c->p.max_iter;
        a.status = st;
        a.active = active;
        launch_density(c, a, grid, tok);
    } else {
        DensArgs<double> a;
        a.tree = tr;
        a.pm = wsa<double4>(c, "pm64", (size_t)s->n);
        a.h = s->h;
        a.rho = (double *)rho;
        a.omega = (double *)omega;
        a.nneigh = nneigh;
        a.iters = iters;
        a.dnn = wsa<double>(c, "dnn64", (size_t)s->capacity);
        a.hmax_new = hmax_new;
        a.pre = pre;
        a.m0 = c->p.m0;
        a.hfact = c->p.hfact;
        a.m0_pi = c->p.m0 / kPi;
        a.hfact3 = c->p.hfact * c->p.hfact * c->p.hfact;
        a.tol = c->p.tol_h;
        a.tol_take = std::sqrt(c->p.tol_h);
        a.hlim = hlim;
        a.max_iter = c->p.max_iter;
        a.status = st;
        a.active = active;
        launch_density(c, a, grid, tok);
    }
    APR_LAUNCHED(c);
    int rc = set_hmax_new(c, hmax_new);  // cells' and tree nodes' h_max for the force search
    if (rc) return rc;
    c->dens_n = s->n;
    return APR_OK;
}

}  // namespace apr
