// Equation of state and the hydrodynamic force sum (grad-h SPH with a
// per-particle artificial viscosity; the paper runs Phantom's compressible
// SPH with an adiabatic or vertically isothermal EOS, Sec. 3 and appendix A):
//   a_a = -sum_b m_b [A_ab F_ab(h_a) + B_ab F_ab(h_b)] rhat_ab
//   du_a/dt = sum_b m_b A_ab (v_ab . rhat) F_ab(h_a)
//   A_ab = (P_a + q^a_ab)/(Omega_a rho_a^2),  B_ab = (P_b + q^b_ab)/(Omega_b rho_b^2)
//   q^a_ab = -1/2 rho_a vsig_a (v_ab . rhat) if v_ab . rhat < 0 else 0,
//   vsig_a = alpha c_a + beta |v_ab . rhat|
//   F_ab(h) = f'(r/h)/(pi h^4) for r < 2h else 0, f' of the M4 or the
//   Wendland C2 kernel (a template parameter)
// over pairs b != a with r < 2 max(h_a, h_b); r = 0 pairs add nothing.
// With Pt = P/(Omega rho^2) and G = 1/(Omega rho) per particle:
//   A_ab = Pt_a - 1/2 G_a vsig_a (v.rhat) for approaching pairs, else Pt_a.
#include "gather.hpp"
#include "sph_kernel.hpp"

namespace apr {

Tree make_tree(apr_ctx *c, const apr_state *s);

namespace {

template <class T>
struct FStageCap;
template <>
struct FStageCap<float> {
    static constexpr int value = 384;
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

// f'(q) of kernel K (0 <= q <= 2)
template <class T, int K>
__device__ inline T kern_df(T q)
{
    T f, df, d2f;
    Kern<K>::template eval<T, 1>(q, f, df, d2f);
    return df;
}

// The force sum as a gather: staged arrays pm, vh = (v, 1/h), th = (Pt, G, c, 0).
template <class T, int K>
struct ForceOp {
    static constexpr int NS = 3;
    static constexpr int SK = 2, SC = 3;  // th.w carries the staged slot
    static constexpr bool EXACT = true;
    using V = vec4_t<T>;
    const V *pm, *vh, *th;
    T *ax, *ay, *az, *dudt, *vsig;
    float *divv;
    int32_t *npair = nullptr;
    const uint8_t *act = nullptr;
    double m0;
    T alpha, beta;
    __device__ V load(int k, int64_t i) const { return k == 0 ? pm[i] : (k == 1 ? vh[i] : th[i]); }
    struct Acc {
        apr::Acc<T> x, y, z, u, dv;
        T vs, hi, hi2, hi4;
    };
    __device__ void init(Acc &A, const V *own) const
    {
        A.x.zero();
        A.y.zero();
        A.z.zero();
        A.u.zero();
        A.dv.zero();
        A.vs = alpha * own[2].z;
        A.hi = own[0].w;
        A.hi2 = A.hi * A.hi;
        A.hi4 = A.hi2 * A.hi2;
    }
    __device__ void pair(Acc &A, const V *own, T dx, T dy, T dz, T r2, const V *nb) const
    {
        T hb = nb[0].w, hb2 = hb * hb;
        bool ina = r2 * A.hi2 < T(4);
        bool inb = r2 * hb2 < T(4);
        T rinv = prsqrt(r2);
        T r = r2 * rinv;
        T Fa = ina ? kern_df<T, K>(r * A.hi) * A.hi4 : T(0);
        T Fb = inb ? kern_df<T, K>(r * hb) * (hb2 * hb2) : T(0);
        T vdr = ((own[1].x - nb[1].x) * dx + (own[1].y - nb[1].y) * dy +
                 (own[1].z - nb[1].z) * dz) * rinv;
        T Aa = own[2].x, Bb = nb[2].x;
        if (vdr < T(0)) {
            T vsa = alpha * own[2].z - beta * vdr;
            T vsb = alpha * nb[2].z - beta * vdr;
            Aa = own[2].x - T(0.5) * own[2].y * vsa * vdr;
            Bb = nb[2].x - T(0.5) * nb[2].y * vsb * vdr;
            A.vs = A.vs > vsa ? A.vs : vsa;
        }
        T mb = nb[1].w;
        T term = mb * (Aa * Fa + Bb * Fb) * rinv;
        A.x.add(-term * dx);
        A.y.add(-term * dy);
        A.z.add(-term * dz);
        A.u.add(mb * Aa * vdr * Fa);
        A.dv.add(mb * vdr * Fa);
    }
    __device__ void finish(Acc &A, int64_t i, const V *own, bool write) const
    {
        A.x.template reduce<kLanes>();
        A.y.template reduce<kLanes>();
        A.z.template reduce<kLanes>();
        A.u.template reduce<kLanes>();
        A.dv.template reduce<kLanes>();
        T vs = max4(A.vs);
        if (!write) return;
        double sc = m0 / kPi;
        ax[i] = (T)(sc * A.x.value());
        ay[i] = (T)(sc * A.y.value());
        az[i] = (T)(sc * A.z.value());
        dudt[i] = (T)(sc * A.u.value());
        if (vsig) vsig[i] = vs;
        // div v_a = -(1/(Omega_a rho_a)) sum_b m_b v_ab . grad_a W_ab(h_a)
        divv[i] = (float)(-(double)own[2].y * sc * A.dv.value());
    }
};

template <class T, int K, bool REST>
__global__ __launch_bounds__(kSearchThreads, kBlocksPerCU<T>) void k_forces(Tree tr,
                                                                             ForceOp<T, K> op,
                                                                             CandList pre,
                                                                             int32_t *status,
                                                                             int64_t first)
{
    gather_pairs<T, ForceOp<T, K>, FStageCap<T>::value, REST>(tr, op, pre, status,
                                                              ST_FORCE_DIRECT, first);
}

template <class T, int K>
void launch_forces(apr_ctx *c, const Tree &tr, const CandList &pre, int64_t n, int64_t grid,
                   int tok, void *ax, void *ay, void *az, void *dudt, void *vsig, float *divv,
                   const uint8_t *active, int32_t *npair)
{
    using V = vec4_t<T>;
    const bool f32 = std::is_same<T, float>::value;
    ForceOp<T, K> op;
    op.pm = wsa<V>(c, f32 ? "pm32" : "pm64", (size_t)n);
    op.vh = wsa<V>(c, f32 ? "vh32" : "vh64", (size_t)n);
    op.th = wsa<V>(c, f32 ? "th32" : "th64", (size_t)n);
    op.ax = (T *)ax;
    op.ay = (T *)ay;
    op.az = (T *)az;
    op.dudt = (T *)dudt;
    op.vsig = (T *)vsig;
    op.divv = divv;
    op.act = active;
    op.npair = npair;
    op.m0 = c->p.m0;
    op.alpha = (T)c->p.av_alpha;
    op.beta = (T)c->p.av_beta;
    hipLaunchKernelGGL((k_forces<T, K, false>), dim3((unsigned)grid), dim3(kSearchThreads), 0,
                       c->stream, tr, op, pre, c->d_status, (int64_t)0);
    prof_end(c, tok);  // the timed pass: the REST launch is nearly always empty
    hipLaunchKernelGGL((k_forces<T, K, true>), dim3(kRestGrid), dim3(kSearchThreads), 0,
                       c->stream, tr, op, pre, c->d_status, grid);
}

template <class T>
void launch_forces(apr_ctx *c, const Tree &tr, const CandList &pre, int64_t n, int64_t grid,
                   int tok, void *ax, void *ay, void *az, void *dudt, void *vsig, float *divv,
                   const uint8_t *active, int32_t *npair)
{
    if (c->p.kernel == APR_KERNEL_WC2)
        launch_forces<T, kWC2>(c, tr, pre, n, grid, tok, ax, ay, az, dudt, vsig, divv, active,
                                npair);
    else
        launch_forces<T, kM4>(c, tr, pre, n, grid, tok, ax, ay, az, dudt, vsig, divv, active,
                               npair);
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
           void *ay, void *az, void *dudt, void *vsig, bool hmax_fresh, const uint8_t *active,
           int32_t *npair)
{
    if (c->cells_n != s->n) return fail(c, APR_ERR_INVALID, "apr_build_cells first");
    if (!rho || !omega || !ax || !ay || !az || !dudt)
        return fail(c, APR_ERR_INVALID, "null output");
    int64_t n = s->n;
    const int64_t grid = c->node_grid[0];
    const apr_params &p = c->p;
    if (p.eos == APR_EOS_ADIABATIC && !s->u) return fail(c, APR_ERR_INVALID, "u is required");
    // the force search needs the supports of the h the state holds now
    int rc = hmax_fresh ? APR_OK : cells_hmax_from(c, s->h, n);
    if (rc) return rc;
    rc = eos_pack(c, s, rho, omega);
    if (rc) return rc;
    Tree tr = make_tree(c, s);
    float *divv = wsa<float>(c, "divv", (size_t)n);
    if (!divv) return fail(c, APR_ERR_HIP, "workspace");
    CandList pre;
    rc = cand_pre(c, tr, true, 2.0, &pre, active);
    if (rc) return rc;
    int tok = prof_begin(c, APR_PROF_FORCES);
    if (p.precision == APR_FP32)
        launch_forces<float>(c, tr, pre, n, grid, tok, ax, ay, az, dudt, vsig, divv, active,
                             npair);
    else
        launch_forces<double>(c, tr, pre, n, grid, tok, ax, ay, az, dudt, vsig, divv, active,
                              npair);
    APR_LAUNCHED(c);
    c->force_n = n;
    c->divv_n = n;
    return APR_OK;
}

}  // namespace apr
