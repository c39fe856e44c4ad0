// Density and smoothing length: the h-rho Newton iteration of every particle
// (the paper defers to Phantom's iterative solve, Sec. 2.2):
//   rho_a = sum_b m_b W(r_ab, h_a)  (b = a included),  h_a = hfact (m_a/rho_a)^(1/3),
//   F(h) = rho_sum(h) - m_a (hfact/h)^3,  F'(h) = sum_b m_b dW/dh + 3 m_a hfact^3/h^4,
//   Omega_a = 1 + h_a/(3 rho_a) sum_b m_b dW_ab/dh_a.
// Newton stops when |dh| < tol h; the h reported is the one the last sums
// were taken at.  If F' <= 0 the step is h_fact (m/rho_sum)^(1/3); every step
// is clamped to [h/2, 2h].
//
// M4 kernel, W = f(q)/(pi h^3), q = r/h:
//   f  = 1 - 3/2 q^2 + 3/4 q^3 (q < 1),  1/4 (2-q)^3 (1 <= q < 2)
//   3f + q f' = 3 - 15/2 q^2 + 9/2 q^3 (q < 1),  3/2 (2-q)^2 (1-q) (1 <= q < 2)
// so dW/dh = -(3f + q f')/(pi h^4).  Sums carry the normalised mass 2^-level;
// m0/pi is applied once in FP64.
//
// Pair arithmetic in T (float: cell-relative coordinates, Kahan-compensated
// sums; double: the same code in FP64).  The Newton update and its
// convergence test are FP64 in both forms.
//
// One workgroup (4 wavefronts) per target cell; each wavefront serves 4
// sub-blocks of 4 targets with 16 lanes per target.  If a target's 2h
// outgrows the staged radius the workgroup searches and stages again with
// the larger radius (bounded: h at most doubles per Newton step, max_iter).
#include "search.hpp"

namespace apr {

namespace {

constexpr float kSigma = 1.1f;  // staged radius margin over 2 h_max

template <class T>
struct StageCap;
template <>
struct StageCap<float> {
    static constexpr int value = 2560;
};
template <>
struct StageCap<double> {
    static constexpr int value = 1280;
};

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
    double m0, hfact, tol;
    int max_iter;
    int32_t *status;
};

// f and 3f + q f' of the M4 kernel, branch-free in q.
template <class T>
__device__ inline void m4_fg(T q, T &f, T &g)
{
    T q2 = q * q;
    T t = T(2) - q;
    T t2 = t * t;
    T fi = T(1) - T(1.5) * q2 + T(0.75) * q2 * q;
    T gi = T(3) - T(7.5) * q2 + T(4.5) * q2 * q;
    T fo = T(0.25) * t2 * t;
    T go = T(1.5) * t2 * (T(1) - q);
    bool inner = q < T(1);
    f = inner ? fi : fo;
    g = inner ? gi : go;
}

// Per-lane partial sums of one Newton evaluation.
template <class T>
struct DSum {
    Acc<T> w, d;   // sum m f, sum m (3f + q f')
    int nn, nzero;
    T dmin;
    __device__ void zero()
    {
        w.zero();
        d.zero();
        nn = 0;
        nzero = 0;
        dmin = T(3.0e38);
    }
    __device__ void pair(T dx, T dy, T dz, T m, T R2, T hinv)
    {
        T r2 = dx * dx + dy * dy + dz * dz;
        if (r2 < R2) {
            T r = sqrt(r2);
            T f, g;
            m4_fg<T>(r * hinv, f, g);
            w.add(m * f);
            d.add(m * g);
            nn += 1;
            if (r2 > T(0)) dmin = dmin < r ? dmin : r;
            else nzero += 1;
        }
    }
    __device__ void reduce16()
    {
        w.reduce16();
        d.reduce16();
        nn = wsum16(nn);
        nzero = wsum16(nzero);
        dmin = wmin16(dmin);
    }
};

template <class T>
__global__ __launch_bounds__(kSearchThreads) void k_density(DensArgs<T> a)
{
    using V = vec4_t<T>;
    constexpr int STAGE = StageCap<T>::value;
    __shared__ int32_t sA[kCandCap], sB[kCandCap];
    __shared__ V stg[STAGE];
    __shared__ uint16_t sub[kWaves][kSubCap];
    __shared__ int s_ncand, s_nstg, s_direct, s_ovf;
    __shared__ double s_red[kWaves];

    const Tree &tr = a.tree;
    int64_t cell = xcd_swizzle(blockIdx.x, gridDim.x);
    if (cell >= tr.hdr->ncells) return;
    const Geo tg = tr.lev[0][cell];
    const int32_t s0 = tr.cs[cell];
    const int cnt = tr.cs[cell + 1] - s0;
    const int w = threadIdx.x / kWave, lane = lane_id(), grp = lane >> 4, j = lane & 15;
    if (threadIdx.x == 0) s_ovf = 0;

    // per lane: the target of its group in each of the wave's 4 sub-blocks
    double hreg[4];
    int itc[4];
    bool done[4];
    double hmy = 0.0;
#pragma unroll
    for (int sb = 0; sb < 4; ++sb) {
        int t = 16 * w + 4 * sb + grp;
        bool v = t < cnt;
        hreg[sb] = v ? a.h[s0 + t] : 0.0;
        itc[sb] = 0;
        done[sb] = !v;
        hmy = fmax(hmy, hreg[sb]);
    }
    {
        double m = hmy;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, kWave));
        if (lane == 0) s_red[w] = m;
    }
    __syncthreads();
    double R = 0.0;
    for (int k = 0; k < kWaves; ++k) R = fmax(R, s_red[k]);
    R *= 2.0 * (double)kSigma;
    const T ex = (T)tg.ex, ey = (T)tg.ey, ez = (T)tg.ez;

    // each new search follows at least one Newton step of a pending target,
    // so max_iter + 1 rounds always finish every target
    for (int round = 0; round < a.max_iter + 2; ++round) {
        // ---- 1. candidate cells
        if (w == 0) {
            int ovf = 0;
            int nc = traverse(tr, tg, R, false, sA, sB, &ovf);
            if (lane == 0) {
                s_ncand = nc;
                if (ovf) s_ovf = 1;
            }
        }
        __syncthreads();
        const int nc = s_ncand;
        const T R2c = (T)(R * R);
        // ---- 2. stage candidates within R of the target cell box: count, scan, write
        for (int pass = 0; pass < 2; ++pass) {
            if (pass == 1 && s_direct) break;
            for (int ci = w; ci < nc; ci += kWaves) {
                int cc = sA[ci];
                int32_t b0 = tr.cs[cc], bn = tr.cs[cc + 1] - b0;
                double sh[3];
                cell_shift(tr.lev[0][cc], tg, tr.box, sh);
                bool hit = false;
                V p;
                if (lane < bn) {
                    p = a.pm[b0 + lane];
                    p.x = p.x + (T)sh[0];
                    p.y = p.y + (T)sh[1];
                    p.z = p.z + (T)sh[2];
                    hit = pt_box_d2<T>(p.x, p.y, p.z, T(0), T(0), T(0), ex, ey, ez) < R2c;
                }
                uint64_t m = __ballot(hit);
                if (pass == 0) {
                    if (lane == 0) sB[ci] = __popcll(m);
                } else if (hit) {
                    stg[sB[ci] + __popcll(m & lanemask_lt())] = p;
                }
            }
            __syncthreads();
            if (pass == 0) {
                if (w == 0) {
                    int tot = wave_excl_scan_lds(sB, nc);
                    if (lane == 0) {
                        s_nstg = tot;
                        s_direct = tot > STAGE;
                    }
                }
                __syncthreads();
            }
        }
        const bool direct = s_direct;
        const int nstg = s_nstg;

        // ---- 3. per sub-block: candidate list, Newton
        double needR = 0.0;
        for (int sb = 0; sb < 4; ++sb) {
            int t = 16 * w + 4 * sb + grp;
            bool valid = t < cnt;
            // the wave skips sub-blocks whose targets are all done
            if (!__any(!done[sb])) continue;
            V tp;
            if (valid) tp = a.pm[s0 + t];
            else { tp.x = T(0); tp.y = T(0); tp.z = T(0); tp.w = T(0); }
            T bigT = T(3.0e38);
            T lox = wmin_groups(valid ? tp.x : bigT), loy = wmin_groups(valid ? tp.y : bigT),
              loz = wmin_groups(valid ? tp.z : bigT);
            T hix = wmax_groups(valid ? tp.x : -bigT), hiy = wmax_groups(valid ? tp.y : -bigT),
              hiz = wmax_groups(valid ? tp.z : -bigT);
            T bcx = T(0.5) * (lox + hix), bcy = T(0.5) * (loy + hiy), bcz = T(0.5) * (loz + hiz);
            T bex = T(0.5) * (hix - lox), bey = T(0.5) * (hiy - loy), bez = T(0.5) * (hiz - loz);
            double h = hreg[sb];
            double ma = valid ? a.m0 * (double)tp.w : 0.0;

            bool need_list = true, sub_direct = direct;
            double Rs = 0.0;
            int nsub = 0;
            while (true) {
                if (need_list) {
                    double hm = wmax_groups(done[sb] ? 0.0 : h);
                    Rs = 2.0 * (double)kSigma * hm;
                    if (Rs > R) {  // candidate set too small: search again
                        needR = fmax(needR, Rs);
                        break;
                    }
                    sub_direct = direct;
                    if (!direct) {
                        // list the staged candidates within Rs of the sub-block box
                        T Rs2 = (T)(Rs * Rs);
                        nsub = 0;
                        wave_sync();  // the previous list is no longer read
                        for (int base = 0; base < nstg; base += kWave) {
                            int idx = base + lane;
                            bool hit = false;
                            if (idx < nstg) {
                                V p = stg[idx];
                                hit = pt_box_d2<T>(p.x, p.y, p.z, bcx, bcy, bcz, bex, bey, bez) < Rs2;
                            }
                            uint64_t m = __ballot(hit);
                            int pos = nsub + __popcll(m & lanemask_lt());
                            if (hit && pos < kSubCap) sub[w][pos] = (uint16_t)idx;
                            nsub += __popcll(m);
                        }
                        if (nsub > kSubCap) sub_direct = true;
                        wave_sync();
                    }
                    need_list = false;
                }
                // one Newton evaluation for the 4 targets
                T hf = (T)h;
                T hinv = T(1) / hf;
                T R2 = T(4) * hf * hf;
                DSum<T> S;
                S.zero();
                if (!sub_direct) {
                    for (int k = j; k < nsub; k += kGroup) {
                        V p = stg[sub[w][k]];
                        S.pair(tp.x - p.x, tp.y - p.y, tp.z - p.z, p.w, R2, hinv);
                    }
                } else {
                    // from global memory: every particle of every candidate cell
                    for (int ci = 0; ci < nc; ++ci) {
                        int cc = sA[ci];
                        int32_t b0 = tr.cs[cc], bn = tr.cs[cc + 1] - b0;
                        double sh[3];
                        cell_shift(tr.lev[0][cc], tg, tr.box, sh);
                        T sx = (T)sh[0], sy = (T)sh[1], sz = (T)sh[2];
                        for (int k = j; k < bn; k += kGroup) {
                            V p = a.pm[b0 + k];
                            S.pair(tp.x - (p.x + sx), tp.y - (p.y + sy), tp.z - (p.z + sz), p.w,
                                   R2, hinv);
                        }
                    }
                }
                S.reduce16();
                // FP64 Newton step (all 16 lanes of a group agree)
                double W = S.w.value(), D = S.d.value();
                double hh = (double)hf;
                double rhos = a.m0 * W / (kPi * hh * hh * hh);
                double drho = -a.m0 * D / (kPi * hh * hh * hh * hh);
                double q3 = a.hfact / hh;
                double rhoh = ma * q3 * q3 * q3;
                double F = rhos - rhoh, dF = drho + 3.0 * rhoh / hh;
                double hn = dF > 0.0 ? hh - F / dF : a.hfact * cbrt(ma / rhos);
                hn = fmin(fmax(hn, 0.5 * hh), 2.0 * hh);
                bool conv = fabs(hn - hh) < a.tol * hh;
                if (!done[sb]) {
                    itc[sb] += 1;
                    bool last = conv || itc[sb] >= a.max_iter;
                    if (last) {
                        done[sb] = true;
                        if (j == 0) {
                            int64_t i = s0 + t;
                            a.h[i] = hh;
                            a.rho[i] = (T)rhos;
                            a.omega[i] = (T)(1.0 - D / (3.0 * W));
                            if (a.nneigh) a.nneigh[i] = S.nn;
                            if (a.iters) a.iters[i] = itc[sb];
                            if (a.dnn)
                                a.dnn[i] = S.nzero >= 2 ? T(0)
                                           : (S.dmin >= T(3.0e38) ? T(__builtin_huge_val()) : S.dmin);
                            if (!conv) atomicAdd(&a.status[ST_NOCONV], 1);
                        }
                        hreg[sb] = hh;
                    } else {
                        hreg[sb] = hn;
                        h = hn;
                    }
                }
                if (!__any(!done[sb])) break;
                // a pending target's support now reaches past the listed radius?
                bool grow = !done[sb] && 2.0 * h > Rs;
                if (__any(grow)) need_list = true;
            }
        }
        // ---- 4. search again with a larger radius if a sub-block needs it
        {
            double m = needR;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, kWave));
            __syncthreads();
            if (lane == 0) s_red[w] = m;
            __syncthreads();
            double need = 0.0;
            for (int k = 0; k < kWaves; ++k) need = fmax(need, s_red[k]);
            if (need <= 0.0) break;
            R = fmax(need, 1.25 * R);
        }
    }

    // ---- new h_max of the cell for the force search
    {
        double m = 0.0;
#pragma unroll
        for (int sb = 0; sb < 4; ++sb) m = fmax(m, hreg[sb]);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, kWave));
        __syncthreads();
        if (lane == 0) s_red[w] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            double hm = 0.0;
            for (int k = 0; k < kWaves; ++k) hm = fmax(hm, s_red[k]);
            a.hmax_new[cell] = f_up(hm);
            if (s_ovf) atomicOr(&a.status[ST_OVERFLOW], 1);
        }
    }
}

__global__ void k_set_cell_hmax(const Hdr *hdr, const float *hmax_new, Geo *cells,
                                int64_t bound)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= bound || c >= hdr->ncells) return;
    cells[c].hmax = hmax_new[c];
}

}  // namespace

Tree make_tree(apr_ctx *c)
{
    Tree t;
    t.hdr = cell_hdr(c);
    t.cs = cell_start(c);
    for (int k = 0; k <= kMaxLev; ++k) t.lev[k] = k <= c->nlev ? cell_level(c, k) : nullptr;
    t.nlev = c->nlev;
    t.box = make_box(c->p);
    return t;
}

int density(apr_ctx *c, apr_state *s, void *rho, void *omega, int32_t *nneigh, int32_t *iters)
{
    if (c->cells_n != s->n) return fail(c, APR_ERR_INVALID, "apr_build_cells first");
    if (!rho || !omega) return fail(c, APR_ERR_INVALID, "rho and omega are required");
    int64_t cb = c->cells_bound;
    float *hmax_new = wsa<float>(c, "hmax_new", (size_t)cb);
    int32_t *st = c->d_status;
    Tree tr = make_tree(c);
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
        a.m0 = c->p.m0;
        a.hfact = c->p.hfact;
        a.tol = c->p.tol_h;
        a.max_iter = c->p.max_iter;
        a.status = st;
        hipLaunchKernelGGL(k_density<float>, dim3((unsigned)cb), dim3(kSearchThreads), 0,
                           c->stream, a);
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
        a.m0 = c->p.m0;
        a.hfact = c->p.hfact;
        a.tol = c->p.tol_h;
        a.max_iter = c->p.max_iter;
        a.status = st;
        hipLaunchKernelGGL(k_density<double>, dim3((unsigned)cb), dim3(kSearchThreads), 0,
                           c->stream, a);
    }
    prof_end(c, tok);
    APR_LAUNCHED(c);
    hipLaunchKernelGGL(k_set_cell_hmax, dim3((unsigned)ceil_div(cb, 256)), dim3(256), 0,
                       c->stream, cell_hdr(c), hmax_new, cell_level(c, 0), cb);
    APR_LAUNCHED(c);
    int rc = refit_hmax_from_cells(c);
    if (rc) return rc;
    c->dens_n = s->n;
    return APR_OK;
}

}  // namespace apr
