// Kick-drift-kick leapfrog (FP64), point-mass (sink) gravity and the Courant
// timestep.  The paper integrates with its host code's individual-timestep
// scheme; this is the standard global-step KDK.
#include <mutex>

#include "common.hpp"

namespace apr {

namespace {

// The step's opening half-kick, v += dtk a (and u += dtk du/dt), then the
// drift x += dt v (wrapped into a periodic box), in one pass.  With divv (the
// velocity divergence of the last force evaluation) the smoothing length is
// predicted from the continuity equation, dh/dt = (h/3) div v, as the Newton
// guess of the next density pass: h *= exp(dt D / 3), the factor kept in
// [0.8, 1.25].  D = div v, or with the divergence of the force evaluation
// before (divv_prev) the two-step extrapolation D = div v + w (div v -
// divv_prev), w = dt / (2 dt_last), which centres it on the new step.  With
// hfac the factor is stored there instead, for a split/merge pass to come
// first (the pass works with the h of the last density pass).
__global__ void k_kick_drift(int64_t n, double *x, double *y, double *z, double *vx, double *vy,
                             double *vz, double *u, const double *ax, const double *ay,
                             const double *az, const double *dudt, double *h, const float *divv,
                             const float *divv_prev, double w, double dtk, double dt, Box b,
                             double *hfac)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v[3] = {vx[i] + dtk * ax[i], vy[i] + dtk * ay[i], vz[i] + dtk * az[i]};
    vx[i] = v[0];
    vy[i] = v[1];
    vz[i] = v[2];
    if (u && dudt) u[i] += dtk * dudt[i];
    if (divv) {
        double D = (double)divv[i];
        if (divv_prev) D += w * (D - (double)divv_prev[i]);
        const double f = fmin(fmax(exp(dt * D / 3.0), 0.8), 1.25);
        if (hfac) hfac[i] = f;
        else h[i] *= f;
    }
    double *p[3] = {x, y, z};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double xn = p[k][i] + dt * v[k];
        if (b.periodic) {
            double hi = b.lo[k] + b.L[k];
            if (xn >= hi) xn -= b.L[k];
            else if (xn < b.lo[k]) xn += b.L[k];
        }
        p[k][i] = xn;
    }
}

constexpr int kMaxSinks = 16;
struct Sinks {
    int n;
    double G;
    double x[kMaxSinks][3], m[kMaxSinks], eps2[kMaxSinks];
};

// With vx non-null it also applies the step's closing half-kick with the new
// accelerations, v += kdt a, u += kdt du/dt.  Individual timesteps: only the
// particles act flags (if given) are touched, and with bin given the
// half-kick is each particle's own, kdt = dt_max 2^-bin / 2.
template <class T>
__global__ void k_total_accel(int64_t n, const double *x, const double *y, const double *z,
                              const T *hax, const T *hay, const T *haz, const T *hdu, Sinks S,
                              double *ax, double *ay, double *az, double *dudt, double kdt,
                              double *vx, double *vy, double *vz, double *u, const uint8_t *act,
                              const int8_t *bin, double dt_max)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (act && !act[i]) return;
    if (bin) kdt = 0.5 * ldexp(dt_max, -(int)bin[i]);
    double gx = (double)hax[i], gy = (double)hay[i], gz = (double)haz[i];
    for (int s = 0; s < S.n; ++s) {
        double dx = x[i] - S.x[s][0], dy = y[i] - S.x[s][1], dz = z[i] - S.x[s][2];
        double d2 = dx * dx + dy * dy + dz * dz + S.eps2[s];
        double inv3 = 1.0 / (d2 * sqrt(d2));
        double f = S.G * S.m[s] * inv3;
        gx -= f * dx;
        gy -= f * dy;
        gz -= f * dz;
    }
    ax[i] = gx;
    ay[i] = gy;
    az[i] = gz;
    if (dudt) dudt[i] = (double)hdu[i];
    if (vx) {
        vx[i] += kdt * gx;
        vy[i] += kdt * gy;
        vz[i] += kdt * gz;
        if (u && dudt) u[i] += kdt * (double)hdu[i];
    }
}

template <class T>
__global__ __launch_bounds__(256) void k_dt_partial(int64_t n, const double *h, const T *vsig,
                                                    double *part)
{
    __shared__ double s[256];
    double m = __builtin_huge_val();
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        double v = (double)vsig[i];
        if (v > 0.0) m = fmin(m, h[i] / v);
    }
    s[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] = fmin(s[threadIdx.x], s[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// out = C min(part[0..np)) (C = 1: the minimum itself)
__global__ __launch_bounds__(256) void k_dt_final(const double *part, int np, double C,
                                                  double *out)
{
#pragma clang fp contract(off)
    __shared__ double s[256];
    double m = __builtin_huge_val();
    for (int i = threadIdx.x; i < np; i += 256) m = fmin(m, part[i]);
    s[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] = fmin(s[threadIdx.x], s[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = C * s[0];
}

// h[i] *= hfac[origin[i]]: the deferred prediction after a split/merge pass
// (children take their parent's factor)
__global__ void k_hfac_apply(int64_t n, const int64_t *origin, const double *hfac, double *h)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) h[i] *= hfac[origin[i]];
}

}  // namespace

int kick_drift(apr_ctx *c, apr_state *s, double dtk, double dt, double **hfac_out)
{
    if (!s->ax || !s->ay || !s->az) return fail(c, APR_ERR_INVALID, "state has no acceleration");
    int64_t n = s->n;
    double *u = c->p.eos == APR_EOS_ADIABATIC ? s->u : nullptr;
    const float *divv = c->divv_n == n ? wsa<float>(c, "divv", (size_t)n) : nullptr;
    const float *divv_prev = divv && c->divv_prev_n == n && c->dt_last > 0.0
                                 ? wsa<float>(c, "divv_prev", (size_t)n)
                                 : nullptr;
    const double w = divv_prev ? dt / (2.0 * c->dt_last) : 0.0;
    double *hfac = nullptr;
    if (hfac_out) {
        *hfac_out = nullptr;
        if (divv) {
            hfac = wsa<double>(c, "hfac", (size_t)n);
            if (!hfac) return fail(c, APR_ERR_HIP, "workspace");
            *hfac_out = hfac;
        }
    }
    hipLaunchKernelGGL(k_kick_drift, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, c->stream,
                       n, s->x, s->y, s->z, s->vx, s->vy, s->vz, u, s->ax, s->ay, s->az, s->dudt,
                       s->h, divv, divv_prev, w, dtk, dt, make_box(c->p), hfac);
    APR_LAUNCHED(c);
    c->cells_n = -1;
    c->dt_last = dt;
    return APR_OK;
}

int hfac_apply(apr_ctx *c, apr_state *s, const int64_t *origin, const double *hfac)
{
    const int64_t n = s->n;
    hipLaunchKernelGGL(k_hfac_apply, dim3((unsigned)ceil_div(n > 0 ? n : 1, 256)), dim3(256), 0,
                       c->stream, n, origin, hfac, s->h);
    APR_LAUNCHED(c);
    return APR_OK;
}

int total_accel(apr_ctx *c, apr_state *s, const void *ax, const void *ay, const void *az,
                const void *dudt, const apr_sink *sinks, int nsinks, double kick_dt,
                const uint8_t *active, const int8_t *bin, double dt_max)
{
    if (nsinks < 0 || nsinks > kMaxSinks) return fail(c, APR_ERR_INVALID, "too many sinks");
    if (!s->ax || !s->ay || !s->az) return fail(c, APR_ERR_INVALID, "state has no acceleration");
    Sinks S;
    std::memset(&S, 0, sizeof(S));
    S.n = nsinks;
    S.G = c->p.G;
    for (int k = 0; k < nsinks; ++k) {
        for (int d = 0; d < 3; ++d) S.x[k][d] = sinks[k].x[d];
        S.m[k] = sinks[k].m;
        S.eps2[k] = sinks[k].eps * sinks[k].eps;
    }
    int64_t n = s->n;
    unsigned g = (unsigned)ceil_div(n, 256);
    const bool k = kick_dt != 0.0 || bin;
    double *u = k && c->p.eos == APR_EOS_ADIABATIC ? s->u : nullptr;
    double *vx = k ? s->vx : nullptr, *vy = k ? s->vy : nullptr, *vz = k ? s->vz : nullptr;
    if (c->p.precision == APR_FP32)
        hipLaunchKernelGGL(k_total_accel<float>, dim3(g), dim3(256), 0, c->stream, n, s->x, s->y,
                           s->z, (const float *)ax, (const float *)ay, (const float *)az,
                           (const float *)dudt, S, s->ax, s->ay, s->az, s->dudt, kick_dt, vx, vy,
                           vz, u, active, bin, dt_max);
    else
        hipLaunchKernelGGL(k_total_accel<double>, dim3(g), dim3(256), 0, c->stream, n, s->x,
                           s->y, s->z, (const double *)ax, (const double *)ay,
                           (const double *)az, (const double *)dudt, S, s->ax, s->ay, s->az,
                           s->dudt, kick_dt, vx, vy, vz, u, active, bin, dt_max);
    APR_LAUNCHED(c);
    return APR_OK;
}

int min_timestep(apr_ctx *c, const apr_state *s, const void *vsig, double C, double *dt)
{
    int64_t n = s->n;
    int np = (int)std::min<int64_t>(1024, ceil_div(n, 256));
    double *part = wsa<double>(c, "dt_part", (size_t)np + 1);
    double *out = part + np;
    if (c->p.precision == APR_FP32)
        hipLaunchKernelGGL(k_dt_partial<float>, dim3(np), dim3(256), 0, c->stream, n, s->h,
                           (const float *)vsig, part);
    else
        hipLaunchKernelGGL(k_dt_partial<double>, dim3(np), dim3(256), 0, c->stream, n, s->h,
                           (const double *)vsig, part);
    hipLaunchKernelGGL(k_dt_final, dim3(1), dim3(256), 0, c->stream, part, np, 1.0, out);
    APR_LAUNCHED(c);
    double v = 0.0;
    APR_HIP(c, hipMemcpyAsync(&v, out, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    APR_HIP(c, hipStreamSynchronize(c->stream));
    *dt = C * v;
    return APR_OK;
}

// ---------------------------------------------------- the timestep, allocation-free
// apr_timestep_noalloc keeps the partial minima of its reduction in this
// file-scope device array instead of the context's workspace.  Each GPU holds
// its own copy until the process ends.  On the host, `scratch` names no
// device address: its address on each device is taken once, with that
// device current, by hipGetSymbolAddress (dt_scratch_setup, from
// apr_ctx_create) and only that pointer is passed to kernels.
static __device__ __align__(256) __attribute__((used)) double scratch[kDtParts];

namespace {
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices];
}  // namespace

int dt_scratch_setup(apr_ctx *c)
{
    if (c->device < 0 || c->device >= kMaxDevices)
        return fail(c, APR_ERR_INVALID, "device index beyond the library's table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[c->device]) return APR_OK;
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_check(c, e, "hipGetSymbolAddress(scratch)");
    g_scratch[c->device] = ptr;
    return APR_OK;
}

int min_timestep_noalloc(apr_ctx *c, const apr_state *s, const void *vsig, double C,
                         double *dt_dev)
{
    double *part = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        part = static_cast<double *>(g_scratch[c->device]);
    }
    if (!part) return fail(c, APR_ERR_INVALID, "no timestep scratch on this device");
    const int64_t n = s->n;
    const int np = (int)std::min<int64_t>(kDtParts, ceil_div(n, 256));
    if (c->p.precision == APR_FP32)
        hipLaunchKernelGGL(k_dt_partial<float>, dim3(np), dim3(256), 0, c->stream, n, s->h,
                           (const float *)vsig, part);
    else
        hipLaunchKernelGGL(k_dt_partial<double>, dim3(np), dim3(256), 0, c->stream, n, s->h,
                           (const double *)vsig, part);
    hipLaunchKernelGGL(k_dt_final, dim3(1), dim3(256), 0, c->stream, part, np, C, dt_dev);
    APR_LAUNCHED(c);
    return APR_OK;
}

}  // namespace apr
