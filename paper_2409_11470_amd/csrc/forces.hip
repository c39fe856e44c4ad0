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
    static constexpr int value = 1024;
};
template <>
struct FStageCap<double> {
    static constexpr int value = 512;
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

template <class T>
__device__ inline T m4_df(T q)
{
    T t = T(2) - q;
    T in = q * (T(-3) + T(2.25) * q);
    T out = T(-0.75) * t * t;
    return q < T(1) ? in : out;
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
            T rinv = T(1) / sqrt(r2);
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
    __shared__ uint16_t sub[kWaves][kSubCap];
    __shared__ int s_ncand, s_nstg, s_direct, s_ovf;

    const Tree &tr = a.tree;
    int64_t cell = xcd_swizzle(blockIdx.x, gridDim.x);
    if (cell >= tr.hdr->ncells) return;
    const Geo tg = tr.lev[0][cell];
    const int32_t s0 = tr.cs[cell];
    const int cnt = tr.cs[cell + 1] - s0;
    const int w = threadIdx.x / kWave, lane = lane_id(), grp = lane >> 4, j = lane & 15;
    const double R = 2.0 * (double)tg.hmax;  // targets' own supports

    if (w == 0) {
        int ovf = 0;
        int nc = traverse(tr, tg, R, true, sA, sB, &ovf);
        if (lane == 0) {
            s_ncand = nc;
            s_ovf = ovf;
        }
    }
    __syncthreads();
    const int nc = s_ncand;
    // stage candidates b within max(R, 2 h_b) of the target cell box: count, scan, write
    {
        const T ex = (T)tg.ex, ey = (T)tg.ey, ez = (T)tg.ez;
        const T R2 = (T)(R * R);
        for (int pass = 0; pass < 2; ++pass) {
            if (pass == 1 && s_direct) break;
            for (int ci = w; ci < nc; ci += kWaves) {
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
                    hit = d2 < R2 || d2 * v.w * v.w < T(4);
                }
                uint64_t m = __ballot(hit);
                if (pass == 0) {
                    if (lane == 0) sB[ci] = __popcll(m);
                } else if (hit) {
                    int pos = sB[ci] + __popcll(m & lanemask_lt());
                    spm[pos] = p;
                    svh[pos] = v;
                    sth[pos] = a.th[b0 + lane];
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
    }
    const bool direct = s_direct;
    const int nstg = s_nstg;

    for (int sb = 0; sb < 4; ++sb) {
        int t = 16 * w + 4 * sb + grp;
        bool valid = t < cnt;
        if (!__any(valid)) break;
        V tp, tv, tt;
        if (valid) {
            tp = a.pm[s0 + t];
            tv = a.vh[s0 + t];
            tt = a.th[s0 + t];
        } else {
            tp.x = tp.y = tp.z = tp.w = T(0);
            tv.x = tv.y = tv.z = tv.w = T(0);
            tt.x = tt.y = tt.z = tt.w = T(0);
        }
        T bigT = T(3.0e38);
        T lox = wmin_groups(valid ? tp.x : bigT), loy = wmin_groups(valid ? tp.y : bigT),
          loz = wmin_groups(valid ? tp.z : bigT);
        T hix = wmax_groups(valid ? tp.x : -bigT), hiy = wmax_groups(valid ? tp.y : -bigT),
          hiz = wmax_groups(valid ? tp.z : -bigT);
        T bcx = T(0.5) * (lox + hix), bcy = T(0.5) * (loy + hiy), bcz = T(0.5) * (loz + hiz);
        T bex = T(0.5) * (hix - lox), bey = T(0.5) * (hiy - loy), bez = T(0.5) * (hiz - loz);
        // largest target support in the sub-block
        T hmin_inv = wmin_groups(valid ? tv.w : bigT);
        T Rs = T(2) / hmin_inv;
        T Rs2 = Rs * Rs;
        int nsub = 0;
        bool sub_direct = direct;
        if (!direct) {
            wave_sync();  // the previous sub-block's list is no longer read
            for (int base = 0; base < nstg; base += kWave) {
                int idx = base + lane;
                bool hit = false;
                if (idx < nstg) {
                    V p = spm[idx];
                    T hb_inv = svh[idx].w;
                    T d2 = pt_box_d2<T>(p.x, p.y, p.z, bcx, bcy, bcz, bex, bey, bez);
                    hit = d2 < Rs2 || d2 * hb_inv * hb_inv < T(4);
                }
                uint64_t m = __ballot(hit);
                int pos = nsub + __popcll(m & lanemask_lt());
                if (hit && pos < kSubCap) sub[w][pos] = (uint16_t)idx;
                nsub += __popcll(m);
            }
            if (nsub > kSubCap) sub_direct = true;
            wave_sync();
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
        if (!sub_direct) {
            for (int k = j; k < nsub; k += kGroup) {
                int e = sub[w][k];
                V p = spm[e];
                S.pair(tp.x - p.x, tp.y - p.y, tp.z - p.z, p.w, svh[e], sth[e]);
            }
        } else {
            for (int ci = 0; ci < nc; ++ci) {
                int cc = sA[ci];
                int32_t b0 = tr.cs[cc], bn = tr.cs[cc + 1] - b0;
                double sh[3];
                cell_shift(tr.lev[0][cc], tg, tr.box, sh);
                T sx = (T)sh[0], sy = (T)sh[1], sz = (T)sh[2];
                for (int k = j; k < bn; k += kGroup) {
                    V p = a.pm[b0 + k];
                    S.pair(tp.x - (p.x + sx), tp.y - (p.y + sy), tp.z - (p.z + sz), p.w,
                           a.vh[b0 + k], a.th[b0 + k]);
                }
            }
        }
        S.x.reduce16();
        S.y.reduce16();
        S.z.reduce16();
        S.u.reduce16();
        T vs = wmax16(S.vs);
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
    __syncthreads();
    if (threadIdx.x == 0 && s_ovf) atomicOr(&a.status[ST_OVERFLOW], 1);
}

}  // namespace

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
    Tree tr = make_tree(c);
    unsigned g = (unsigned)ceil_div(n, 256);
    if (p.precision == APR_FP32) {
        float4 *vh = wsa<float4>(c, "vh32", (size_t)n), *th = wsa<float4>(c, "th32", (size_t)n);
        hipLaunchKernelGGL(k_eos<float>, dim3(g), dim3(256), 0, c->stream, n, p.eos, p.cs0,
                           p.q_cs, p.r_ref, p.gamma, s->x, s->y, s->vx, s->vy, s->vz, s->u, s->h,
                           (const float *)rho, (const float *)omega, vh, th);
        int tok = prof_begin(c, APR_PROF_FORCES);
        ForceArgs<float> a;
        a.tree = tr;
        a.pm = wsa<float4>(c, "pm32", (size_t)n);
        a.vh = vh;
        a.th = th;
        a.ax = (float *)ax; a.ay = (float *)ay; a.az = (float *)az;
        a.dudt = (float *)dudt; a.vsig = (float *)vsig;
        a.m0 = p.m0; a.alpha = p.av_alpha; a.beta = p.av_beta;
        a.status = c->d_status;
        hipLaunchKernelGGL(k_forces<float>, dim3((unsigned)cb), dim3(kSearchThreads), 0,
                           c->stream, a);
        prof_end(c, tok);
    } else {
        double4 *vh = wsa<double4>(c, "vh64", (size_t)n),
                *th = wsa<double4>(c, "th64", (size_t)n);
        hipLaunchKernelGGL(k_eos<double>, dim3(g), dim3(256), 0, c->stream, n, p.eos, p.cs0,
                           p.q_cs, p.r_ref, p.gamma, s->x, s->y, s->vx, s->vy, s->vz, s->u, s->h,
                           (const double *)rho, (const double *)omega, vh, th);
        int tok = prof_begin(c, APR_PROF_FORCES);
        ForceArgs<double> a;
        a.tree = tr;
        a.pm = wsa<double4>(c, "pm64", (size_t)n);
        a.vh = vh;
        a.th = th;
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
