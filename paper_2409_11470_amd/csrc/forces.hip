// Equation of state and the hydrodynamic force sum (grad-h SPH with a
// per-particle artificial viscosity; the paper runs Phantom's compressible
// SPH with an adiabatic or vertically isothermal EOS, Sec. 3 and appendix A):
//   a_a = -sum_b m_b [A_ab F_ab(h_a) + B_ab F_ab(h_b)] rhat_ab
//   du_a/dt = sum_b m_b A_ab (v_ab . rhat) F_ab(h_a)
//   A_ab = (P_a + q^a_ab)/(Omega_a rho_a^2),  B_ab = (P_b + q^b_ab)/(Omega_b rho_b^2)
//   q^a_ab = -1/2 rho_a vsig_a (v_ab . rhat) if v_ab . rhat < 0 else 0,
//   vsig_a = alpha c_a + beta |v_ab . rhat|
//   F_ab(h) = f'(r/h)/(pi h^4) for r < 2h else 0,  f' = -3q + 9/4 q^2 (q < 1),
//   -3/4 (2-q)^2 (1 <= q < 2)
// over pairs b != a with r < 2 max(h_a, h_b); r = 0 pairs add nothing.
// With Pt = P/(Omega rho^2) and G = 1/(Omega rho) per particle:
//   A_ab = Pt_a - 1/2 G_a vsig_a (v.rhat) for approaching pairs, else Pt_a.
#include "search.hpp"

namespace apr {

Tree make_tree(apr_ctx *c);

namespace {

template <class T>
struct FStageCap;
template <>
struct FStageCap<float> {
    static constexpr int value = 640;
};
template <>
struct FStageCap<double> {
    static constexpr int value = 320;
};

// Per particle: vh = (vx, vy, vz, 1/h), th = (P/(Omega rho^2), 1/(Omega rho), c, 0).
template <class T>
__global__ void k_eos(int64_t n, int eos, double cs0, double q_cs, double r_ref, double gamma,
                      const double *x, const double *y, const double *vx, const double *vy,
                      const double *vz, const double *u, const double *h, const T *rho,
                      const T *omega, vec4_t<T> *vh, vec4_t<T> *th)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double r = (double)rho[i], om = (double)omega[i];
    double P, c;
    if (eos == APR_EOS_ISOTHERMAL) {
        c = cs0;
        P = cs0 * cs0 * r;
    } else if (eos == APR_EOS_LOCALLY_ISOTHERMAL) {
        double R = sqrt(x[i] * x[i] + y[i] * y[i]);
        c = cs0 * pow(R / r_ref, -q_cs);
        P = c * c * r;
    } else {
        P = (gamma - 1.0) * r * u[i];
        c = sqrt(gamma * P / r);
    }
    vec4_t<T> a, b;
    a.x = (T)vx[i];
    a.y = (T)vy[i];
    a.z = (T)vz[i];
    a.w = (T)(1.0 / h[i]);
    b.x = (T)(P / (om * r * r));
    b.y = (T)(1.0 / (om * r));
    b.z = (T)c;
    b.w = T(0);
    vh[i] = a;
    th[i] = b;
}

template <class T>
struct ForceArgs {
    Tree tree;
    const vec4_t<T> *pm, *vh, *th;
    T *ax, *ay, *az, *dudt, *vsig;
    double m0, alpha, beta;
    int32_t *status;
};

// f'(q) of the M4 kernel, branch-free (0 <= q < 2): -3/4 (2-q)^2 + 3 max(1-q, 0)^2.
template <class T>
__device__ inline T m4_df(T q)
{
    T t = T(2) - q;
    T u = T(1) - q;
    u = u > T(0) ? u : T(0);
    return T(3) * u * u - T(0.75) * t * t;
}

// Per-lane partial sums of the force on one target.
template <class T>
struct FSum {
    Acc<T> x, y, z, u;
    T vs;
    // target data
    T tx, ty, tz, tvx, tvy, tvz, ha_inv2, ha_inv4, ha_inv, Pa, Ga, ca, alpha, beta;
    __device__ void pair(T dx, T dy, T dz, T mb, const vec4_t<T> &v, const vec4_t<T> &tb)
    {
        T r2 = dx * dx + dy * dy + dz * dz;
        T hb_inv2 = v.w * v.w;
        bool ina = r2 * ha_inv2 < T(4);
        bool inb = r2 * hb_inv2 < T(4);
        if ((ina || inb) && r2 > T(0)) {
            T rinv = prsqrt(r2);
            T r = r2 * rinv;
            T Fa = ina ? m4_df<T>(r * ha_inv) * ha_inv4 : T(0);
            T Fb = inb ? m4_df<T>(r * v.w) * (hb_inv2 * hb_inv2) : T(0);
            T vdr = ((tvx - v.x) * dx + (tvy - v.y) * dy + (tvz - v.z) * dz) * rinv;
            T A = Pa, B = tb.x;
            if (vdr < T(0)) {
                T vsa = alpha * ca - beta * vdr;
                T vsb = alpha * tb.z - beta * vdr;
                A = Pa - T(0.5) * Ga * vsa * vdr;
                B = tb.x - T(0.5) * tb.y * vsb * vdr;
                vs = vs > vsa ? vs : vsa;
            }
            T term = mb * (A * Fa + B * Fb) * rinv;
            x.add(-term * dx);
            y.add(-term * dy);
            z.add(-term * dz);
            u.add(mb * A * vdr * Fa);
        }
    }
};

template <class T>
__global__ __launch_bounds__(kSearchThreads) void k_forces(ForceArgs<T> a)
{
    using V = vec4_t<T>;
    constexpr int STAGE = FStageCap<T>::value;
    __shared__ int32_t sA[kCandCap], sB[kCandCap];
    __shared__ V spm[STAGE], svh[STAGE], sth[STAGE];
    __shared__ uint16_t sub[kWaves][STAGE];
    __shared__ uint16_t tls[kCell][kTCap];
    __shared__ int s_ncand, s_total, s_tlen[kCell];

    const Tree &tr = a.tree;
    int64_t cell = xcd_swizzle(blockIdx.x, gridDim.x);
    if (cell >= tr.hdr->ncells) return;
    const Geo tg = tr.lev[0][cell];
    const int32_t s0 = tr.cs[cell];
    const int cnt = tr.cs[cell + 1] - s0;
    const int w = threadIdx.x / kWave, lane = lane_id(), j = lane & 3;
    const int t = 16 * w + (lane >> 2);   // this lane's target (4 lanes each)
    const bool valid = t < cnt;
    uint16_t *mylist = tls[t < kCell ? t : 0];
    const double R = 2.0 * (double)tg.hmax;  // targets' own supports
    const T ex = (T)tg.ex, ey = (T)tg.ey, ez = (T)tg.ez;
    const T R2c = (T)(R * R);

    if (w == 0) {
        int o = 0;
        int ncl = traverse(tr, tg, R, true, sA, sB, &o);
        if (lane == 0) {
            s_ncand = ncl;
            if (o) atomicOr(&a.status[ST_OVERFLOW], 1);
        }
    }
    __syncthreads();
    const int nc = s_ncand;
    // candidates b within max(R, 2 h_b) of the target cell box: count per cell
    for (int ci = w; ci < nc; ci += kWaves) {
        int cc = sA[ci];
        int32_t b0 = tr.cs[cc], bn = tr.cs[cc + 1] - b0;
        double sh[3];
        cell_shift(tr.lev[0][cc], tg, tr.box, sh);
        bool hit = false;
        if (lane < bn) {
            V p = a.pm[b0 + lane];
            T hb = a.vh[b0 + lane].w;
            T d2 = pt_box_d2<T>(p.x + (T)sh[0], p.y + (T)sh[1], p.z + (T)sh[2], T(0), T(0), T(0),
                                ex, ey, ez);
            hit = d2 < R2c || d2 * hb * hb < T(4);
        }
        uint64_t m = __ballot(hit);
        if (lane == 0) sB[ci] = __popcll(m);
    }
    __syncthreads();
    if (w == 0) {
        int tot = wave_excl_scan_lds(sB, nc);
        if (lane == 0) {
            s_total = tot;
            if (tot > STAGE) atomicAdd(&a.status[ST_FORCE_DIRECT], 1);
        }
    }
    __syncthreads();
    const int total = s_total;
    const int nwin = total > STAGE ? (total + STAGE - 1) / STAGE : 1;

    V tp, tv, tt;
    if (valid) {
        tp = a.pm[s0 + t];
        tv = a.vh[s0 + t];
        tt = a.th[s0 + t];
    } else {
        tp.x = tp.y = tp.z = tp.w = T(0);
        tv.x = tv.y = tv.z = T(0);
        tv.w = T(0);
        tt.x = tt.y = tt.z = tt.w = T(0);
    }
    FSum<T> S;
    S.x.zero(); S.y.zero(); S.z.zero(); S.u.zero();
    S.alpha = (T)a.alpha;
    S.beta = (T)a.beta;
    S.tx = tp.x; S.ty = tp.y; S.tz = tp.z;
    S.tvx = tv.x; S.tvy = tv.y; S.tvz = tv.z;
    S.ha_inv = tv.w;
    S.ha_inv2 = tv.w * tv.w;
    S.ha_inv4 = S.ha_inv2 * S.ha_inv2;
    S.Pa = tt.x; S.Ga = tt.y; S.ca = tt.z;
    S.vs = S.alpha * S.ca;
    const bool wave_busy = __any(valid);

    for (int win = 0; win < nwin; ++win) {
        const int w0 = win * STAGE;
        const int nstg = min(STAGE, total - w0);
        if (win > 0) __syncthreads();  // the previous window is no longer read
        // stage the window
        for (int ci = w; ci < nc; ci += kWaves) {
            int o0 = sB[ci], o1 = ci + 1 < nc ? sB[ci + 1] : total;
            if (o1 <= w0 || o0 >= w0 + STAGE || o1 == o0) continue;
            int cc = sA[ci];
            int32_t b0 = tr.cs[cc], bn = tr.cs[cc + 1] - b0;
            double sh[3];
            cell_shift(tr.lev[0][cc], tg, tr.box, sh);
            bool hit = false;
            V p, v;
            if (lane < bn) {
                p = a.pm[b0 + lane];
                v = a.vh[b0 + lane];
                p.x = p.x + (T)sh[0];
                p.y = p.y + (T)sh[1];
                p.z = p.z + (T)sh[2];
                T d2 = pt_box_d2<T>(p.x, p.y, p.z, T(0), T(0), T(0), ex, ey, ez);
                hit = d2 < R2c || d2 * v.w * v.w < T(4);
            }
            uint64_t m = __ballot(hit);
            int off = o0 + __popcll(m & lanemask_lt()) - w0;
            if (hit && off >= 0 && off < STAGE) {
                spm[off] = p;
                svh[off] = v;
                sth[off] = a.th[b0 + lane];
            }
        }
        __syncthreads();
        if (!wave_busy) continue;
        // this target's own pairs: r^2 < 4 max(h_a, h_b)^2
        const T Ra = valid ? T(2) / tv.w : T(0);
        build_lists16<T>(
            nstg, spm, sub[w], &tls[0][0], kTCap, s_tlen,
            [&](int k) {
                V q;
                int tt = 16 * w + k;
                if (tt < cnt) q = a.pm[s0 + tt];
                else { q.x = T(0); q.y = T(0); q.z = T(0); q.w = T(0); }
                return q;
            },
            [&](int k) { return __shfl(Ra, 4 * k, kWave); },
            [&](T d2, T Rs2, int e) {
                T hb = svh[e].w;
                return d2 < Rs2 || d2 * hb * hb < T(4);
            },
            [&](const V &q, T rk, int e) {
                V p = spm[e];
                T hb = svh[e].w;
                T dx = q.x - p.x, dy = q.y - p.y, dz = q.z - p.z;
                T r2 = dx * dx + dy * dy + dz * dz;
                return r2 < rk * rk || r2 * hb * hb < T(4);
            });
        const int tlen = s_tlen[t < kCell ? t : 0];
        if (!valid) continue;
        if (tlen <= kTCap) {
            for (int k = j; k < tlen; k += kLanes) {
                int e = mylist[k];
                V p = spm[e];
                S.pair(tp.x - p.x, tp.y - p.y, tp.z - p.z, p.w, svh[e], sth[e]);
            }
        } else {
            // own list overflowed: walk the whole window
            for (int e = j; e < nstg; e += kLanes) {
                V p = spm[e];
                S.pair(tp.x - p.x, tp.y - p.y, tp.z - p.z, p.w, svh[e], sth[e]);
            }
        }
    }

    S.x.template reduce<kLanes>();
    S.y.template reduce<kLanes>();
    S.z.template reduce<kLanes>();
    S.u.template reduce<kLanes>();
    T vs = max4(S.vs);
    if (valid && j == 0) {
        double sc = a.m0 / kPi;
        int64_t i = s0 + t;
        a.ax[i] = (T)(sc * S.x.value());
        a.ay[i] = (T)(sc * S.y.value());
        a.az[i] = (T)(sc * S.z.value());
        a.dudt[i] = (T)(sc * S.u.value());
        if (a.vsig) a.vsig[i] = vs;
    }
}

}  // namespace

int eos_pack(apr_ctx *c, const apr_state *s, const void *rho, const void *omega)
{
    int64_t n = s->n;
    const apr_params &p = c->p;
    unsigned g = (unsigned)ceil_div(n, 256);
    if (p.precision == APR_FP32) {
        float4 *vh = wsa<float4>(c, "vh32", (size_t)n), *th = wsa<float4>(c, "th32", (size_t)n);
        if (!vh || !th) return fail(c, APR_ERR_HIP, "workspace");
        hipLaunchKernelGGL(k_eos<float>, dim3(g), dim3(256), 0, c->stream, n, p.eos, p.cs0,
                           p.q_cs, p.r_ref, p.gamma, s->x, s->y, s->vx, s->vy, s->vz, s->u, s->h,
                           (const float *)rho, (const float *)omega, vh, th);
    } else {
        double4 *vh = wsa<double4>(c, "vh64", (size_t)n),
                *th = wsa<double4>(c, "th64", (size_t)n);
        if (!vh || !th) return fail(c, APR_ERR_HIP, "workspace");
        hipLaunchKernelGGL(k_eos<double>, dim3(g), dim3(256), 0, c->stream, n, p.eos, p.cs0,
                           p.q_cs, p.r_ref, p.gamma, s->x, s->y, s->vx, s->vy, s->vz, s->u, s->h,
                           (const double *)rho, (const double *)omega, vh, th);
    }
    APR_LAUNCHED(c);
    return APR_OK;
}

int forces(apr_ctx *c, const apr_state *s, const void *rho, const void *omega, void *ax,
           void *ay, void *az, void *dudt, void *vsig)
{
    if (c->cells_n != s->n) return fail(c, APR_ERR_INVALID, "apr_build_cells first");
    if (!rho || !omega || !ax || !ay || !az || !dudt)
        return fail(c, APR_ERR_INVALID, "null output");
    int64_t n = s->n;
    int64_t cb = c->cells_bound;
    const apr_params &p = c->p;
    if (p.eos == APR_EOS_ADIABATIC && !s->u) return fail(c, APR_ERR_INVALID, "u is required");
    // the force search needs the supports of the h the state holds now
    int rc = cells_hmax_from(c, s->h, n);
    if (rc) return rc;
    rc = eos_pack(c, s, rho, omega);
    if (rc) return rc;
    Tree tr = make_tree(c);
    if (p.precision == APR_FP32) {
        int tok = prof_begin(c, APR_PROF_FORCES);
        ForceArgs<float> a;
        a.tree = tr;
        a.pm = wsa<float4>(c, "pm32", (size_t)n);
        a.vh = wsa<float4>(c, "vh32", (size_t)n);
        a.th = wsa<float4>(c, "th32", (size_t)n);
        a.ax = (float *)ax; a.ay = (float *)ay; a.az = (float *)az;
        a.dudt = (float *)dudt; a.vsig = (float *)vsig;
        a.m0 = p.m0; a.alpha = p.av_alpha; a.beta = p.av_beta;
        a.status = c->d_status;
        hipLaunchKernelGGL(k_forces<float>, dim3((unsigned)cb), dim3(kSearchThreads), 0,
                           c->stream, a);
        prof_end(c, tok);
    } else {
        int tok = prof_begin(c, APR_PROF_FORCES);
        ForceArgs<double> a;
        a.tree = tr;
        a.pm = wsa<double4>(c, "pm64", (size_t)n);
        a.vh = wsa<double4>(c, "vh64", (size_t)n);
        a.th = wsa<double4>(c, "th64", (size_t)n);
        a.ax = (double *)ax; a.ay = (double *)ay; a.az = (double *)az;
        a.dudt = (double *)dudt; a.vsig = (double *)vsig;
        a.m0 = p.m0; a.alpha = p.av_alpha; a.beta = p.av_beta;
        a.status = c->d_status;
        hipLaunchKernelGGL(k_forces<double>, dim3((unsigned)cb), dim3(kSearchThreads), 0,
                           c->stream, a);
        prof_end(c, tok);
    }
    APR_LAUNCHED(c);
    c->force_n = n;
    return APR_OK;
}

}  // namespace apr
