// Individual timesteps (paper Sec. 2.5).  Particle a sits in bin k_a and steps
// with dt_max 2^-k_a; a step of dt_max runs 2^K substeps of dt_max 2^-K, K the
// largest bin.  In substep s:
//   - a particle whose own step starts (s a multiple of 2^(K-k)) takes its
//     opening half kick with its own dt;
//   - every particle drifts by the substep;
//   - the particles whose step ends ((s+1) a multiple of 2^(K-k)) are active:
//     the split/merge pass examines only them (random key step 4096 + s),
//     density, forces and sink gravity are taken for them and for what the
//     pass made (the others keep h, rho, Omega, a from their last turn, which
//     their neighbours use), and they take their closing half kick;
//   - an active particle's bin then follows the Courant limit dt_max 2^-k <=
//     c_cfl h / vsig (an integer search), clamped to K within the step (the
//     substep grid is fixed) and to max_bin at its end, and moves to a longer
//     step only where that step starts at this boundary; what the pass made
//     or kept takes bin K (the finest, as the paper asks).
// Each particle's last rho, Omega, vsig and nearest distance live in the
// context ("bn_*", context precision) and are carried through every
// reordering: the cell build's permutation and the pass's origins.
#include "common.hpp"

namespace apr {

namespace {

unsigned g256(int64_t n) { return (unsigned)ceil_div(n > 0 ? n : 1, 256); }

constexpr int kRebuild = 8;  // substeps between full cell builds when nothing splits or merges

// the smallest k >= 0 with dt_max 2^-k <= c_cfl h / vsig, at most kmax
template <class T>
__device__ inline int courant_k(double h, T vs, double dt_max, double c_cfl, int kmax)
{
    const double dtc = c_cfl * h / (double)vs;
    int k = 0;
    while (k < kmax && ldexp(dt_max, -k) > dtc) ++k;
    return k;
}

template <class T>
__global__ void k_bins_init(int64_t n, const double *h, const T *vs, double dt_max, double c_cfl,
                            int kmax, int8_t *bin)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) bin[i] = (int8_t)courant_k<T>(h[i], vs[i], dt_max, c_cfl, kmax);
}

// out[0]: the largest bin; out[1]: 1 if any bin is negative
__global__ void k_max_bin(int64_t n, const int8_t *bin, int32_t *out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int v = i < n ? bin[i] : 0;
    if (v < 0) atomicOr(out + 1, 1);
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const int t = __shfl_xor(v, o, kWave);
        v = v > t ? v : t;
    }
    if (lane_id() == 0 && v > 0) atomicMax(out, v);
}

// Substep s opens: the opening half kick of the particles whose step starts
// (s a multiple of 2^(K-bin)), with their own dt; the drift of every particle
// by the substep (wrapped into a periodic box); act = the particle's step ends
// with this substep ((s+1) a multiple of 2^(K-bin)); made cleared.
__global__ void k_substep_open(int64_t n, const int8_t *bin, int K, int64_t s, double dt_max,
                               double delta, double *x, double *y, double *z, double *vx,
                               double *vy, double *vz, double *u, const double *ax,
                               const double *ay, const double *az, const double *dudt, Box b,
                               uint8_t *act, uint8_t *made)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int bi = bin[i];
    const int64_t stride = (int64_t)1 << (K - bi);
    double v[3] = {vx[i], vy[i], vz[i]};
    if (s % stride == 0) {
        const double kd = 0.5 * ldexp(dt_max, -bi);
        v[0] += kd * ax[i];
        v[1] += kd * ay[i];
        v[2] += kd * az[i];
        vx[i] = v[0];
        vy[i] = v[1];
        vz[i] = v[2];
        if (u) u[i] += kd * dudt[i];
    }
    double *p[3] = {x, y, z};
    for (int k = 0; k < 3; ++k) {
        double xn = p[k][i] + delta * v[k];
        if (b.periodic) {
            const double hi = b.lo[k] + b.L[k];
            if (xn >= hi) xn -= b.L[k];
            else if (xn < b.lo[k]) xn += b.L[k];
        }
        p[k][i] = xn;
    }
    act[i] = (s + 1) % stride == 0 ? 1 : 0;
    made[i] = 0;
}

__global__ void k_or_made(int64_t n, uint8_t *act, const uint8_t *made)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) act[i] = act[i] | made[i];
}

template <class T>
__global__ void k_copy_active(int64_t n, const uint8_t *act, const T *src, T *dst)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && act[i]) dst[i] = src[i];
}

template <class T>
__global__ void k_rebin(int64_t n, const uint8_t *act, const uint8_t *made, int8_t *bin,
                        const double *h, const T *vs, double dt_max, double c_cfl, int K,
                        int64_t s, int kmax_last, int last)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !act[i]) return;
    int k = made[i] ? K : courant_k<T>(h[i], vs[i], dt_max, c_cfl, last ? kmax_last : K);
    if (!last)
        while ((s + 1) % ((int64_t)1 << (K - k))) ++k;
    bin[i] = (int8_t)k;
}

template <class T>
struct Stored {
    T *rho, *om, *vs, *dnn;      // per particle, kept between turns
    T *ax, *ay, *az, *du;        // hydro sums of the active particles (this substep)
};

// The stored arrays keep their first `keep` entries when the capacity grows.
template <class T>
int stored(apr_ctx *c, int64_t cap, int64_t keep, Stored<T> *b)
{
    static const char *nm[8] = {"bn_rho", "bn_om", "bn_vs", "bn_dnn",
                                "bn_ax", "bn_ay", "bn_az", "bn_du"};
    T **p[8] = {&b->rho, &b->om, &b->vs, &b->dnn, &b->ax, &b->ay, &b->az, &b->du};
    for (int k = 0; k < 8; ++k) {
        const size_t kb = k < 4 && keep > 0 ? (size_t)keep * sizeof(T) : 0;
        *p[k] = (T *)ws_keep(c, nm[k], (size_t)cap * sizeof(T) + 256, kb);
        if (!*p[k]) return fail(c, APR_ERR_HIP, "timestep-bin workspace");
    }
    return APR_OK;
}

template <class T>
T *dnn_ws(apr_ctx *c, int64_t n)
{
    return wsa<T>(c, sizeof(T) == 4 ? "dnn32" : "dnn64", (size_t)n);
}

// Up to 8 per-particle arrays (elements of 1, 4 or 8 bytes) permuted together:
// one gather into workspace copies, one copy back.
struct Remap {
    char *a[8], *t[8];
    int es[8];
    int na;
};

template <class E>
__device__ inline void mv(char *dst, int64_t i, const char *src, int64_t j)
{
    reinterpret_cast<E *>(dst)[i] = reinterpret_cast<const E *>(src)[j];
}

__global__ void k_take_all(int64_t n, const int64_t *idx, Remap r)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t j = idx[i];
    for (int k = 0; k < r.na; ++k) {
        if (r.es[k] == 1) mv<uint8_t>(r.t[k], i, r.a[k], j);
        else if (r.es[k] == 4) mv<uint32_t>(r.t[k], i, r.a[k], j);
        else mv<uint64_t>(r.t[k], i, r.a[k], j);
    }
}

__global__ void k_put_all(int64_t n, Remap r)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int k = 0; k < r.na; ++k) {
        if (r.es[k] == 1) mv<uint8_t>(r.a[k], i, r.t[k], i);
        else if (r.es[k] == 4) mv<uint32_t>(r.a[k], i, r.t[k], i);
        else mv<uint64_t>(r.a[k], i, r.t[k], i);
    }
}

template <class T>
int remap_all(apr_ctx *c, int8_t *bin, const Stored<T> &b, uint8_t *act, uint8_t *made,
              const int64_t *idx, int64_t n)
{
    static const char *nm[8] = {"bn_r0", "bn_r1", "bn_r2", "bn_r3",
                                "bn_r4", "bn_r5", "bn_r6", "bn_r7"};
    Remap r;
    r.na = 0;
    auto add = [&](void *p, int es) {
        r.a[r.na] = (char *)p;
        r.t[r.na] = (char *)ws(c, nm[r.na], (size_t)n * es + 256);
        r.es[r.na] = es;
        return r.t[r.na++] != nullptr;
    };
    bool ok = add(bin, 1) && add(act, 1) && (!made || add(made, 1));
    T *arr[4] = {b.rho, b.om, b.vs, b.dnn};
    for (int k = 0; k < 4 && ok; ++k) ok = add(arr[k], (int)sizeof(T));
    if (!ok) return fail(c, APR_ERR_HIP, "timestep-bin workspace");
    hipLaunchKernelGGL(k_take_all, dim3(g256(n)), dim3(256), 0, c->stream, n, idx, r);
    hipLaunchKernelGGL(k_put_all, dim3(g256(n)), dim3(256), 0, c->stream, n, r);
    APR_LAUNCHED(c);
    return APR_OK;
}

template <class T>
int bins_init_t(apr_ctx *c, apr_state *s, int8_t *bin, const apr_sink *sinks, int nsinks,
                double dt_max, double c_cfl, int max_bin)
{
    Stored<T> b;
    int rc = stored<T>(c, s->capacity, 0, &b);
    if (rc) return rc;
    rc = build_cells(c, s, nullptr, false);
    if (rc) return rc;
    const int64_t n = s->n;
    rc = density(c, s, b.rho, b.om, nullptr, nullptr);
    if (rc) return rc;
    APR_HIP(c, hipMemcpyAsync(b.dnn, dnn_ws<T>(c, n), (size_t)n * sizeof(T),
                              hipMemcpyDeviceToDevice, c->stream));
    rc = forces(c, s, b.rho, b.om, b.ax, b.ay, b.az, b.du, b.vs);
    if (rc) return rc;
    rc = total_accel(c, s, b.ax, b.ay, b.az, b.du, sinks, nsinks, 0.0);
    if (rc) return rc;
    hipLaunchKernelGGL(k_bins_init<T>, dim3(g256(n)), dim3(256), 0, c->stream, n, s->h, b.vs,
                       dt_max, c_cfl, max_bin, bin);
    APR_LAUNCHED(c);
    c->bins_n = n;
    return APR_OK;
}

// *K = the largest bin; every bin must lie in 0..max_bin
int bin_range(apr_ctx *c, const apr_state *s, const int8_t *bin, int max_bin, int32_t *K)
{
    int32_t *kmax_dev = wsa<int32_t>(c, "bn_kmax", 2);
    if (!kmax_dev) return fail(c, APR_ERR_HIP, "timestep-bin workspace");
    int32_t kb[2] = {0, 0};
    APR_HIP(c, hipMemsetAsync(kmax_dev, 0, 8, c->stream));
    hipLaunchKernelGGL(k_max_bin, dim3(g256(s->n)), dim3(256), 0, c->stream, s->n, bin, kmax_dev);
    APR_LAUNCHED(c);
    APR_HIP(c, hipMemcpyAsync(kb, kmax_dev, 8, hipMemcpyDeviceToHost, c->stream));
    APR_HIP(c, hipStreamSynchronize(c->stream));
    if (kb[1]) return fail(c, APR_ERR_INVALID, "a negative bin");
    if (kb[0] > max_bin) return fail(c, APR_ERR_INVALID, "a bin above max_bin");
    *K = kb[0];
    return APR_OK;
}

template <class T>
int step_bins_t(apr_ctx *c, apr_state *s, int8_t *bin, const apr_zone *zones, int nzones,
                const apr_sink *sinks, int nsinks, double dt_max, double c_cfl, int max_bin,
                int32_t K, int64_t step, int32_t *nsub_out)
{
    const int64_t cap = s->capacity;
    Stored<T> b;
    int rc = stored<T>(c, cap, s->n, &b);
    if (rc) return rc;
    uint8_t *act = wsa<uint8_t>(c, "bn_act", (size_t)cap);
    uint8_t *made = wsa<uint8_t>(c, "bn_made", (size_t)cap);
    int64_t *idx = wsa<int64_t>(c, "bn_idx", (size_t)cap);
    if (!act || !made || !idx) return fail(c, APR_ERR_HIP, "timestep-bin workspace");
    const int64_t nsub = (int64_t)1 << K;
    const double delta = ldexp(dt_max, -K);
    const Box box = make_box(c->p);
    double *u = c->p.eos == APR_EOS_ADIABATIC ? s->u : nullptr;
    for (int64_t sub = 0; sub < nsub; ++sub) {
        int64_t n = s->n;
        bool changed = false;  // the split/merge pass changed the particle set
        hipLaunchKernelGGL(k_substep_open, dim3(g256(n)), dim3(256), 0, c->stream, n, bin, K,
                           sub, dt_max, delta, s->x, s->y, s->z, s->vx, s->vy, s->vz, u, s->ax,
                           s->ay, s->az, s->dudt, box, act, made);
        APR_LAUNCHED(c);
        if (nzones > 0) {
            if (c->p.nn_cap > 0.0) {
                // every particle's last nearest distance, for the split cap
                APR_HIP(c, hipMemcpyAsync(dnn_ws<T>(c, n), b.dnn, (size_t)n * sizeof(T),
                                          hipMemcpyDeviceToDevice, c->stream));
                c->dens_n = n;
            }
            int64_t ns = 0, nm = 0, nsp = 0;
            rc = split_merge(c, s, zones, nzones, step * 4096 + sub, 0, &ns, &nm, &nsp, act,
                             idx, made);
            if (rc) return rc;
            if (ns + nm > 0) {
                changed = true;
                n = s->n;
                rc = remap_all<T>(c, bin, b, act, nullptr, idx, n);
                if (rc) return rc;
                hipLaunchKernelGGL(k_or_made, dim3(g256(n)), dim3(256), 0, c->stream, n, act,
                                   made);
                APR_LAUNCHED(c);
            }
        }
        // a substep whose pass changed nothing keeps the cells and refits them
        // to the drifted positions (the particles of a cell move together);
        // every kRebuild-th substep sorts again, so that they stay compact.
        // Not in a periodic box: a particle the drift wrapped to the far side
        // would stretch its cell across the box, and the cell's one periodic
        // image shift would then be wrong for part of its particles
        if (sub % kRebuild == 0 || changed || c->cells_n != n || c->p.periodic) {
            rc = build_cells(c, s, idx, true);
            if (rc) return rc;
            rc = remap_all<T>(c, bin, b, act, made, idx, n);
            if (rc) return rc;
        } else {
            rc = refit_cells(c, s);
            if (rc) return rc;
        }
        rc = density(c, s, b.rho, b.om, nullptr, nullptr, act);
        if (rc) return rc;
        hipLaunchKernelGGL(k_copy_active<T>, dim3(g256(n)), dim3(256), 0, c->stream, n, act,
                           dnn_ws<T>(c, n), b.dnn);
        APR_LAUNCHED(c);
        rc = forces(c, s, b.rho, b.om, b.ax, b.ay, b.az, b.du, b.vs, false, act);
        if (rc) return rc;
        rc = total_accel(c, s, b.ax, b.ay, b.az, b.du, sinks, nsinks, 0.0, act, bin, dt_max);
        if (rc) return rc;
        hipLaunchKernelGGL(k_rebin<T>, dim3(g256(n)), dim3(256), 0, c->stream, n, act, made, bin,
                           s->h, b.vs, dt_max, c_cfl, K, sub, max_bin, (int)(sub + 1 == nsub));
        APR_LAUNCHED(c);
    }
    if (nsub_out) *nsub_out = (int32_t)nsub;
    return APR_OK;
}

// clears in_bins on every way out
struct InBins {
    apr_ctx *c;
    explicit InBins(apr_ctx *cc) : c(cc) { c->in_bins = true; }
    ~InBins() { c->in_bins = false; }
};

}  // namespace

int bins_init(apr_ctx *c, apr_state *s, int8_t *bin, const apr_sink *sinks, int nsinks,
              double dt_max, double c_cfl, int max_bin)
{
    c->bins_n = -1;
    int rc = c->p.precision == APR_FP32
                 ? bins_init_t<float>(c, s, bin, sinks, nsinks, dt_max, c_cfl, max_bin)
                 : bins_init_t<double>(c, s, bin, sinks, nsinks, dt_max, c_cfl, max_bin);
    return rc;
}

int step_bins(apr_ctx *c, apr_state *s, int8_t *bin, const apr_zone *zones, int nzones,
              const apr_sink *sinks, int nsinks, double dt_max, double c_cfl, int max_bin,
              int64_t step, int32_t *nsub)
{
    if (c->bins_n != s->n)
        return fail(c, APR_ERR_INVALID, "apr_bins_init first (or the state was reordered since)");
    int32_t K = 0;
    int rc = bin_range(c, s, bin, max_bin, &K);   // changes nothing on failure
    if (rc) return rc;
    {
        InBins guard(c);
        rc = c->p.precision == APR_FP32
                 ? step_bins_t<float>(c, s, bin, zones, nzones, sinks, nsinks, dt_max, c_cfl,
                                      max_bin, K, step, nsub)
                 : step_bins_t<double>(c, s, bin, zones, nzones, sinks, nsinks, dt_max, c_cfl,
                                       max_bin, K, step, nsub);
    }
    c->bins_n = rc ? -1 : s->n;
    return rc;
}

}  // namespace apr
