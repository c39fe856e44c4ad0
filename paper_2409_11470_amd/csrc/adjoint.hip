// Adjoint (vector-Jacobian product) of the density and force sums with
// respect to particle positions and masses, with the smoothing length
// implicit (h solves the h-rho relation).  Gather-only: every target
// accumulates the derivatives of all terms that depend on its own variables.
//
// Pair (p, q), r = x_p - x_q, rhat = r/|r|, vdr = (v_p - v_q).rhat:
//   a_p gets  -m_q (A_p F_p + A_q F_q) rhat,   du_p gets m_q A_p vdr F_p,
//   a_q gets  +m_p (A_q F_q + A_p F_p) rhat,   du_q gets m_p A_q vdr F_q,
// with F_p = W'(r, h_p), A_p = Pt_p - 1/2 (alpha c_p - beta vdr) vdr G_p for
// approaching pairs (else Pt_p), Pt = P/(Omega rho^2), G = 1/(Omega rho).
// With cotangents abar, ubar the pair's share of the loss is
//   L_pq = (A_p F_p + A_q F_q) (m_p abar_q - m_q abar_p).rhat
//        + vdr (ubar_p m_q A_p F_p + ubar_q m_p A_q F_q),
// symmetric in p and q.
// Pass 1 (pairs): dL_pq/d(x_p, m_p, Pt_p, G_p, c_p, h_p) and
//   S2_p = sum_q m_q d2W/dh2(r, h_p).
// Pass 2 (per particle, FP64): the EOS (P, c from rho and u or R), Omega =
//   1 + h D/(3 rho) with D = sum m dW/dh, and h = hfact (m/rho)^(1/3) turn these
//   into a total rho cotangent; the implicit density gives c = rhobar/Omega and
//   the self-mass term rhobar (rho/m)(1 - 1/Omega).
// Pass 3 (pairs): x_p gets (c_p m_q F_p + c_q m_p F_q + D_p m_q H_p +
//   D_q m_p H_q) rhat with H = d2W/dr dh and Dbar = Omegabar h/(3 rho);
//   m_p gets sum_q c_q W(r, h_q) + Dbar_q dW/dh(r, h_q), self term included.
#include "gather.hpp"
#include "sph_kernel.hpp"

namespace apr {

Tree make_tree(apr_ctx *c, const apr_state *s);
int eos_pack(apr_ctx *c, const apr_state *s, const void *rho, const void *omega);

namespace {

// Staging windows (entries) and workgroups per CU of the adjoint gathers.
// The FP32 density adjoint runs four per CU, its window sized so that its
// LDS stays within the 40 KB that four allow (it needs at most 128 VGPRs
// anyway): more windows per cell, but the extra wavefronts hide more latency
// (refined box: its 768-entry windows at three per CU were 5 % slower; 8M
// disc 13.3 -> 12.8 ms).  The force adjoint keeps the compiler's choice: at
// four per CU it spills 48 B per lane, 2.4 GB of writes per launch on the 8M
// disc, for no gain there.  FP64: the compiler's choice (a bound spills
// hundreds of bytes per lane and is slower).
template <class T>
struct VJPStage;
template <>
struct VJPStage<float> {
    static constexpr int force = 384, dens = 512;
    static constexpr int force_blocks = 1, dens_blocks = 4;
};
template <>
struct VJPStage<double> {
    static constexpr int force = 256, dens = 512;
    static constexpr int force_blocks = 1, dens_blocks = 1;
};

template <class T, int K>
struct ForceVJP {
    static constexpr int NS = 4;
    static constexpr int SK = 2, SC = 3;  // th.w carries the staged slot
    static constexpr bool EXACT = false;
    int32_t *npair = nullptr;
    using V = vec4_t<T>;
    const V *pm, *vh, *th, *cot;
    T alpha, beta;
    T *out[9];  // xbar[3], mbar, Ptbar, Gbar, cbar, hbar, S2
    const uint8_t *act = nullptr;  // every target
    __device__ V load(int k, int64_t i) const
    {
        return k == 0 ? pm[i] : (k == 1 ? vh[i] : (k == 2 ? th[i] : cot[i]));
    }
    struct Acc {
        apr::Acc<T> a[9];
    };
    __device__ void init(Acc &A, const V *) const
    {
        for (int k = 0; k < 9; ++k) A.a[k].zero();
    }
    __device__ void pair(Acc &A, const V *own, T dx, T dy, T dz, T r2, const V *nb) const
    {
        T rinv = prsqrt(r2);
        T r = r2 * rinv;
        T rx = dx * rinv, ry = dy * rinv, rz = dz * rinv;
        T hp = own[0].w, hq = nb[0].w;
        T qp = r * hp, qq = r * hq;
        bool inp = qp < T(2), inq = qq < T(2);
        T fp, dfp, d2fp, fq, dfq, d2fq;
        Kern<K>::template eval<T, 2>(inp ? qp : T(2), fp, dfp, d2fp);
        Kern<K>::template eval<T, 2>(inq ? qq : T(2), fq, dfq, d2fq);
        T hp2 = hp * hp, hp4 = hp2 * hp2, hp5 = hp4 * hp;
        T hq2 = hq * hq, hq4 = hq2 * hq2, hq5 = hq4 * hq;
        T Fp = inp ? dfp * hp4 : T(0), Fpr = inp ? d2fp * hp5 : T(0);
        T Fq = inq ? dfq * hq4 : T(0), Fqr = inq ? d2fq * hq5 : T(0);
        T Fph = inp ? -(qp * d2fp + T(4) * dfp) * hp5 : T(0);
        T vx = own[1].x - nb[1].x, vy = own[1].y - nb[1].y, vz = own[1].z - nb[1].z;
        T vdr = vx * rx + vy * ry + vz * rz;
        T Ptp = own[2].x, Gp = own[2].y, cp = own[2].z;
        T Ptq = nb[2].x, Gq = nb[2].y, cq = nb[2].z;
        bool appr = vdr < T(0);
        T Ap = Ptp, Aq = Ptq, dAp = T(0), dAq = T(0), avp = T(0);
        if (appr) {
            avp = T(-0.5) * (alpha * cp - beta * vdr) * vdr;
            Ap = Ptp + avp * Gp;
            Aq = Ptq + T(-0.5) * (alpha * cq - beta * vdr) * vdr * Gq;
            dAp = T(-0.5) * (alpha * cp - T(2) * beta * vdr) * Gp;
            dAq = T(-0.5) * (alpha * cq - T(2) * beta * vdr) * Gq;
        }
        T mp = own[1].w, mq = nb[1].w;
        T ubp = own[3].w, ubq = nb[3].w;
        T Sx = mp * nb[3].x - mq * own[3].x, Sy = mp * nb[3].y - mq * own[3].y,
          Sz = mp * nb[3].z - mq * own[3].z;
        T s = Sx * rx + Sy * ry + Sz * rz;
        T G = Ap * Fp + Aq * Fq;
        T E = ubp * mq * Ap * Fp + ubq * mp * Aq * Fq;
        T dGr = Ap * Fpr + Aq * Fqr;
        T dEr = ubp * mq * Ap * Fpr + ubq * mp * Aq * Fqr;
        T dGv = Fp * dAp + Fq * dAq;
        T dEv = ubp * mq * Fp * dAp + ubq * mp * Fq * dAq;
        T c1 = dGr * s + vdr * dEr;
        T c2 = G * rinv;
        T c3 = (dGv * s + E + vdr * dEv) * rinv;
        T cr = c1 - c2 * s - c3 * vdr;
        A.a[0].add(cr * rx + c2 * Sx + c3 * vx);
        A.a[1].add(cr * ry + c2 * Sy + c3 * vy);
        A.a[2].add(cr * rz + c2 * Sz + c3 * vz);
        T aqr = nb[3].x * rx + nb[3].y * ry + nb[3].z * rz;
        A.a[3].add(G * aqr + vdr * ubq * Aq * Fq);
        T w = s + vdr * ubp * mq;
        T LA = Fp * w;
        A.a[4].add(LA);
        if (appr) {
            A.a[5].add(LA * avp);
            A.a[6].add(LA * T(-0.5) * alpha * vdr * Gp);
        }
        A.a[7].add(Ap * w * Fph);
        if (inp) A.a[8].add(mq * (T(12) * fp + T(8) * qp * dfp + qp * qp * d2fp) * hp5);
    }
    __device__ void finish(Acc &A, int64_t i, const V *, bool write) const
    {
        for (int k = 0; k < 9; ++k) A.a[k].template reduce<kLanes>();
        if (write)
            for (int k = 0; k < 9; ++k) out[k][i] = (T)A.a[k].value();
    }
};

template <class T, int K>
struct DensVJP {
    static constexpr int NS = 2;
    static constexpr int SK = 1, SC = 2;  // dv.z carries the staged slot
    static constexpr bool EXACT = false;
    int32_t *npair = nullptr;
    using V = vec4_t<T>;
    const V *pm, *dv;  // dv = (c = rhobar/Omega, Dbar, 0, 1/h)
    const double *xb[3], *mb;
    double scx, scm;   // m0/pi, 1/pi
    T *xbar[3], *mbar;
    const uint8_t *act = nullptr;  // every target
    __device__ V load(int k, int64_t i) const { return k == 0 ? pm[i] : dv[i]; }
    struct Acc {
        apr::Acc<T> a[4];
    };
    __device__ void init(Acc &A, const V *) const
    {
        for (int k = 0; k < 4; ++k) A.a[k].zero();
    }
    __device__ void pair(Acc &A, const V *own, T dx, T dy, T dz, T r2, const V *nb) const
    {
        T rinv = prsqrt(r2);
        T r = r2 * rinv;
        T hp = own[0].w, hq = nb[0].w;
        T qp = r * hp, qq = r * hq;
        bool inp = qp < T(2), inq = qq < T(2);
        T fp, dfp, d2fp, fq, dfq, d2fq;
        Kern<K>::template eval<T, 2>(inp ? qp : T(2), fp, dfp, d2fp);
        Kern<K>::template eval<T, 2>(inq ? qq : T(2), fq, dfq, d2fq);
        T hp2 = hp * hp, hp4 = hp2 * hp2, hp5 = hp4 * hp;
        T hq2 = hq * hq, hq3 = hq2 * hq, hq4 = hq2 * hq2, hq5 = hq4 * hq;
        T Fp = inp ? dfp * hp4 : T(0), Fq = inq ? dfq * hq4 : T(0);
        T Hp = inp ? -(qp * d2fp + T(4) * dfp) * hp5 : T(0);
        T Hq = inq ? -(qq * d2fq + T(4) * dfq) * hq5 : T(0);
        T Wq = inq ? fq * hq3 : T(0);
        T Whq = inq ? -(T(3) * fq + qq * dfq) * hq4 : T(0);
        T mp = own[1].w, mq = nb[1].w;
        T cp = own[1].x, Dp = own[1].y, cq = nb[1].x, Dq = nb[1].y;
        T coef = (cp * mq * Fp + cq * mp * Fq + Dp * mq * Hp + Dq * mp * Hq) * rinv;
        A.a[0].add(coef * dx);
        A.a[1].add(coef * dy);
        A.a[2].add(coef * dz);
        A.a[3].add(cq * Wq + Dq * Whq);
    }
    __device__ void finish(Acc &A, int64_t i, const V *own, bool write) const
    {
        for (int k = 0; k < 4; ++k) A.a[k].template reduce<kLanes>();
        if (!write) return;
        T hp = own[0].w;
        // self pair (r = 0): c W(0, h) + Dbar dW/dh(0, h), with f(0) of the kernel
        double self = Kern<K>::f0 * ((double)own[1].x * (double)(hp * hp * hp) -
                                     3.0 * (double)own[1].y * (double)(hp * hp * hp * hp));
        for (int k = 0; k < 3; ++k) xbar[k][i] = (T)(xb[k][i] + scx * A.a[k].value());
        mbar[i] = (T)(mb[i] + scm * (A.a[3].value() + self));
    }
};

template <class T, int K, bool REST>
__global__ __launch_bounds__(kSearchThreads, VJPStage<T>::force_blocks) void k_vjp_force(Tree tr, ForceVJP<T, K> op,
                                                              CandList pre, int32_t *status,
                                                              int64_t first)
{
    gather_pairs<T, ForceVJP<T, K>, VJPStage<T>::force, REST>(tr, op, pre, status, -1, first);
}

template <class T, int K, bool REST>
__global__ __launch_bounds__(kSearchThreads, VJPStage<T>::dens_blocks) void k_vjp_dens(Tree tr, DensVJP<T, K> op,
                                                             CandList pre, int32_t *status,
                                                             int64_t first)
{
    gather_pairs<T, DensVJP<T, K>, VJPStage<T>::dens, REST>(tr, op, pre, status, -1, first);
}

template <class T>
__global__ void k_pack_cot(int64_t n, const T *ax, const T *ay, const T *az, const T *du,
                           vec4_t<T> *cot)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    vec4_t<T> v;
    v.x = ax ? ax[i] : T(0);
    v.y = ay ? ay[i] : T(0);
    v.z = az ? az[i] : T(0);
    v.w = du ? du[i] : T(0);
    cot[i] = v;
}

template <class T>
struct FPtrs {
    const T *p[9];
};

struct LocalArgs {
    int64_t n;
    const double *x, *y, *u, *h;
    const int8_t *level;
    double m0, hfact, cs0, q_cs, r_ref, gamma;
    double f0;  // f(0) of the kernel (the self pair)
    int eos, has_force;
};

// Per particle, FP64: chain rules of the EOS, Omega and h(rho, m); writes the
// partial position / mass cotangents and (c, Dbar, 0, 1/h) for pass 3.
template <class T>
__global__ void k_vjp_local(LocalArgs a, const T *rho, const T *omega, const T *rho_bar,
                            const T *h_bar, FPtrs<T> f, double *xb0, double *xb1, double *xb2, double *mb,
                            vec4_t<T> *dv)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const double pi = kPi;
    double r = (double)rho[i], om = (double)omega[i], h = a.h[i];
    double m = ldexp(a.m0, -(int)a.level[i]);
    double P, c, R = 0.0;
    if (a.eos == APR_EOS_ISOTHERMAL) {
        c = a.cs0;
        P = c * c * r;
    } else if (a.eos == APR_EOS_LOCALLY_ISOTHERMAL) {
        R = sqrt(a.x[i] * a.x[i] + a.y[i] * a.y[i]);
        c = a.cs0 * pow(R / a.r_ref, -a.q_cs);
        P = c * c * r;
    } else {
        P = (a.gamma - 1.0) * r * a.u[i];
        c = sqrt(a.gamma * P / r);
    }
    double Pt = P / (om * r * r), G = 1.0 / (om * r);
    double sc = a.m0 / pi;
    double xb[3] = {0.0, 0.0, 0.0}, mbar = 0.0, Ptb = 0.0, Gb = 0.0, cb = 0.0, hb = 0.0, S2 = 0.0;
    if (a.has_force) {
        for (int k = 0; k < 3; ++k) xb[k] = sc * (double)f.p[k][i];
        mbar = (double)f.p[3][i] / pi;
        Ptb = sc * (double)f.p[4][i];
        Gb = sc * (double)f.p[5][i];
        cb = sc * (double)f.p[6][i];
        hb = sc * (double)f.p[7][i];
        S2 = sc * (double)f.p[8][i];
    }
    S2 += 12.0 * a.f0 * m / (pi * h * h * h * h * h);  // self term of sum_q m_q d2W/dh2
    if (h_bar) hb += (double)h_bar[i];
    double Ob = -(Ptb * Pt + Gb * G) / om;
    double rb = (rho_bar ? (double)rho_bar[i] : 0.0) - (2.0 * Ptb * Pt + Gb * G) / r;
    double Pb = Ptb / (om * r * r);
    if (a.eos == APR_EOS_ISOTHERMAL) {
        rb += Pb * a.cs0 * a.cs0;
    } else if (a.eos == APR_EOS_LOCALLY_ISOTHERMAL) {
        rb += Pb * c * c;
        double ct = cb + 2.0 * c * r * Pb;
        if (R > 0.0) {
            xb[0] += ct * (-a.q_cs) * c * a.x[i] / (R * R);
            xb[1] += ct * (-a.q_cs) * c * a.y[i] / (R * R);
        }
    } else {
        rb += Pb * (a.gamma - 1.0) * a.u[i];
    }
    double D = 3.0 * r * (om - 1.0) / h;
    double Db = Ob * h / (3.0 * r);
    hb += Ob * D / (3.0 * r) + Db * S2;
    rb += -Ob * (om - 1.0) / r;
    // h = hfact (m / rho)^(1/3)
    rb += -hb * h / (3.0 * r);
    mbar += hb * h / (3.0 * m);
    // implicit density: d rho_a / d m_a has the extra (rho/m)(1 - 1/Omega)
    mbar += rb * (r / m) * (1.0 - 1.0 / om);
    xb0[i] = xb[0];
    xb1[i] = xb[1];
    xb2[i] = xb[2];
    mb[i] = mbar;
    vec4_t<T> o;
    o.x = (T)(rb / om);
    o.y = (T)Db;
    o.z = T(0);
    o.w = (T)(1.0 / h);
    dv[i] = o;
}

template <class T, int K>
int vjp_t(apr_ctx *c, const apr_state *s, const void *rho, const void *omega,
          const void *rho_bar, const void *h_bar, const void *ax_bar, const void *ay_bar, const void *az_bar,
          const void *dudt_bar, void *xbar, void *ybar, void *zbar, void *mbar)
{
    using V = vec4_t<T>;
    const int64_t n = s->n, grid = c->node_grid[0];
    const apr_params &p = c->p;
    bool has_force = ax_bar || ay_bar || az_bar || dudt_bar;
    int rc = cells_hmax_from(c, s->h, n);
    if (rc) return rc;
    rc = eos_pack(c, s, rho, omega);
    if (rc) return rc;
    const bool f32 = std::is_same<T, float>::value;
    const V *pm = (const V *)ws(c, f32 ? "pm32" : "pm64", n * sizeof(V) + 256);
    const V *vh = (const V *)ws(c, f32 ? "vh32" : "vh64", n * sizeof(V) + 256);
    const V *th = (const V *)ws(c, f32 ? "th32" : "th64", n * sizeof(V) + 256);
    Tree tr = make_tree(c, s);
    CandList pre;
    rc = cand_pre(c, tr, true, 2.0, &pre);
    if (rc) return rc;
    unsigned g = (unsigned)ceil_div(n, 256);
    static const char *fn[9] = {"vf0", "vf1", "vf2", "vf3", "vf4", "vf5", "vf6", "vf7", "vf8"};
    T *fout[9];
    for (int k = 0; k < 9; ++k) {
        fout[k] = wsa<T>(c, fn[k], (size_t)n);
        if (!fout[k]) return fail(c, APR_ERR_HIP, "vjp workspace");
    }
    if (has_force) {
        V *cot = wsa<V>(c, f32 ? "cot32" : "cot64", (size_t)n);
        if (!cot) return fail(c, APR_ERR_HIP, "vjp workspace");
        hipLaunchKernelGGL(k_pack_cot<T>, dim3(g), dim3(256), 0, c->stream, n,
                           (const T *)ax_bar, (const T *)ay_bar, (const T *)az_bar,
                           (const T *)dudt_bar, cot);
        ForceVJP<T, K> op;
        op.pm = pm;
        op.vh = vh;
        op.th = th;
        op.cot = cot;
        op.alpha = (T)p.av_alpha;
        op.beta = (T)p.av_beta;
        for (int k = 0; k < 9; ++k) op.out[k] = fout[k];
        hipLaunchKernelGGL((k_vjp_force<T, K, false>), dim3((unsigned)grid), dim3(kSearchThreads), 0,
                           c->stream, tr, op, pre, c->d_status, (int64_t)0);
        hipLaunchKernelGGL((k_vjp_force<T, K, true>), dim3(kRestGrid), dim3(kSearchThreads), 0,
                           c->stream, tr, op, pre, c->d_status, grid);
        APR_LAUNCHED(c);
    }
    FPtrs<T> fp;
    for (int k = 0; k < 9; ++k) fp.p[k] = fout[k];
    double *xb[3] = {wsa<double>(c, "vxb0", (size_t)n), wsa<double>(c, "vxb1", (size_t)n),
                     wsa<double>(c, "vxb2", (size_t)n)};
    double *mb = wsa<double>(c, "vmb", (size_t)n);
    V *dv = wsa<V>(c, f32 ? "vdv32" : "vdv64", (size_t)n);
    if (!xb[0] || !xb[1] || !xb[2] || !mb || !dv) return fail(c, APR_ERR_HIP, "vjp workspace");
    LocalArgs la;
    la.n = n;
    la.x = s->x;
    la.y = s->y;
    la.u = s->u;
    la.h = s->h;
    la.level = s->level;
    la.m0 = p.m0;
    la.hfact = p.hfact;
    la.cs0 = p.cs0;
    la.q_cs = p.q_cs;
    la.r_ref = p.r_ref;
    la.gamma = p.gamma;
    la.f0 = Kern<K>::f0;
    la.eos = p.eos;
    la.has_force = has_force;
    hipLaunchKernelGGL(k_vjp_local<T>, dim3(g), dim3(256), 0, c->stream, la, (const T *)rho,
                       (const T *)omega, (const T *)rho_bar, (const T *)h_bar, fp, xb[0], xb[1], xb[2], mb, dv);
    APR_LAUNCHED(c);
    DensVJP<T, K> dop;
    dop.pm = pm;
    dop.dv = dv;
    for (int k = 0; k < 3; ++k) dop.xb[k] = xb[k];
    dop.mb = mb;
    dop.scx = p.m0 / kPi;
    dop.scm = 1.0 / kPi;
    dop.xbar[0] = (T *)xbar;
    dop.xbar[1] = (T *)ybar;
    dop.xbar[2] = (T *)zbar;
    dop.mbar = (T *)mbar;
    hipLaunchKernelGGL((k_vjp_dens<T, K, false>), dim3((unsigned)grid), dim3(kSearchThreads), 0,
                       c->stream, tr, dop, pre, c->d_status, (int64_t)0);
    hipLaunchKernelGGL((k_vjp_dens<T, K, true>), dim3(kRestGrid), dim3(kSearchThreads), 0, c->stream,
                       tr, dop, pre, c->d_status, grid);
    APR_LAUNCHED(c);
    return APR_OK;
}

}  // namespace

int vjp(apr_ctx *c, const apr_state *s, const void *rho, const void *omega, const void *rho_bar,
        const void *h_bar, const void *ax_bar, const void *ay_bar, const void *az_bar, const void *dudt_bar,
        void *xbar, void *ybar, void *zbar, void *mbar)
{
    if (c->cells_n != s->n) return fail(c, APR_ERR_INVALID, "apr_build_cells first");
    if (!rho || !omega || !xbar || !ybar || !zbar || !mbar)
        return fail(c, APR_ERR_INVALID, "null argument");
    if (c->p.eos == APR_EOS_ADIABATIC && !s->u) return fail(c, APR_ERR_INVALID, "u is required");
    int tok = prof_begin(c, APR_PROF_VJP);
    const bool f32 = c->p.precision == APR_FP32, wc2 = c->p.kernel == APR_KERNEL_WC2;
    auto run = f32 ? (wc2 ? vjp_t<float, kWC2> : vjp_t<float, kM4>)
                   : (wc2 ? vjp_t<double, kWC2> : vjp_t<double, kM4>);
    int rc = run(c, s, rho, omega, rho_bar, h_bar, ax_bar, ay_bar, az_bar, dudt_bar, xbar, ybar,
                 zbar, mbar);
    prof_end(c, tok);
    return rc;
}

}  // namespace apr
