// C ABI of libapr.so: argument checks, the context and its workspace, and
// the order of kernel launches for each call.  No exceptions cross the ABI.
#include <cstdio>
#include <new>

#include "common.hpp"

namespace apr {

int fail(apr_ctx *c, int code, const std::string &msg)
{
    if (c) c->err = msg;
    return code;
}

int fail(apr_ctx *c, int code, const char *msg)
{
    if (c) c->err.assign(msg);  // within the reserved capacity: no allocation
    return code;
}

int hip_check(apr_ctx *c, hipError_t e, const char *what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(c, APR_ERR_HIP, m);
}

void *ws(apr_ctx *c, const char *name, size_t bytes)
{
    for (auto &b : c->bufs) {
        if (b.name == name) {
            if (b.bytes >= bytes) return b.p;
            // growing: queued kernels may still use the old buffer
            if (hipStreamSynchronize(c->stream) != hipSuccess) return nullptr;
            if (hipFree(b.p) != hipSuccess) return nullptr;
            b.p = nullptr;
            size_t nb = bytes + bytes / 4;
            if (hipMalloc(&b.p, nb) != hipSuccess) {
                b.bytes = 0;
                c->err = std::string("workspace allocation failed: ") + name;
                return nullptr;
            }
            b.bytes = nb;
            return b.p;
        }
    }
    apr_ctx::Buf b;
    b.name = name;
    b.bytes = bytes;
    if (hipMalloc(&b.p, bytes) != hipSuccess) {
        c->err = std::string("workspace allocation failed: ") + name;
        return nullptr;
    }
    c->bufs.push_back(b);
    return b.p;
}

void *ws_peek(apr_ctx *c, const char *name, size_t bytes)
{
    for (auto &b : c->bufs)
        if (b.name == name) return b.bytes >= bytes ? b.p : nullptr;
    return nullptr;
}

void *ws_keep(apr_ctx *c, const char *name, size_t bytes, size_t keep)
{
    for (auto &b : c->bufs) {
        if (b.name != name) continue;
        if (b.bytes >= bytes) return b.p;
        // growing: the first `keep` bytes move to the new buffer
        void *np = nullptr;
        size_t nb = bytes + bytes / 4;
        if (hipMalloc(&np, nb) != hipSuccess) {
            c->err = std::string("workspace allocation failed: ") + name;
            return nullptr;
        }
        if (keep > 0 &&
            hipMemcpyAsync(np, b.p, std::min(keep, b.bytes), hipMemcpyDeviceToDevice,
                           c->stream) != hipSuccess)
            return nullptr;
        if (hipStreamSynchronize(c->stream) != hipSuccess) return nullptr;
        if (hipFree(b.p) != hipSuccess) return nullptr;
        b.p = np;
        b.bytes = nb;
        return b.p;
    }
    return ws(c, name, bytes);
}

int prof_begin(apr_ctx *c, int idx)
{
    if (!c->prof || !((c->prof_mask >> idx) & 1u)) return -1;
    apr_ctx::EvPair e;
    if (!c->ev_free.empty()) {
        e = c->ev_free.back();
        c->ev_free.pop_back();
    } else if (hipEventCreate(&e.a) != hipSuccess || hipEventCreate(&e.b) != hipSuccess) {
        return -1;
    }
    e.idx = idx;
    if (hipEventRecord(e.a, c->stream) != hipSuccess) {
        c->ev_free.push_back(e);
        return -1;
    }
    c->ev_used.push_back(e);
    return (int)c->ev_used.size() - 1;
}

void prof_end(apr_ctx *c, int token)
{
    if (token < 0) return;
    (void)hipEventRecord(c->ev_used[token].b, c->stream);
}

}  // namespace apr

using namespace apr;

namespace {

int check_state(apr_ctx *c, const apr_state *s, bool need_vel)
{
    if (!c) return APR_ERR_INVALID;
    if (!s) return fail(c, APR_ERR_INVALID, "null state");
    if (s->n <= 0 || s->n > s->capacity) return fail(c, APR_ERR_INVALID, "bad n / capacity");
    // cell starts and particle slots are 32-bit
    if (s->capacity > (int64_t)INT32_MAX)
        return fail(c, APR_ERR_INVALID, "capacity above 2^31 - 1 particles");
    if (!s->x || !s->y || !s->z || !s->h || !s->level || !s->id)
        return fail(c, APR_ERR_INVALID, "state needs x, y, z, h, level, id");
    if (need_vel && (!s->vx || !s->vy || !s->vz))
        return fail(c, APR_ERR_INVALID, "state needs vx, vy, vz");
    return APR_OK;
}

int check_params(const apr_params *p, std::string &why)
{
    if (p->precision != APR_FP32 && p->precision != APR_FP64) return why = "precision", 1;
    if (p->eos < 0 || p->eos > 2) return why = "eos", 1;
    if (p->kernel != APR_KERNEL_M4 && p->kernel != APR_KERNEL_WC2) return why = "kernel", 1;
    if (!(p->hfact > 0) || !(p->tol_h > 0) || p->max_iter < 1 || p->max_iter > 1000)
        return why = "hfact/tol/max_iter", 1;
    if (!(p->m0 > 0)) return why = "m0", 1;
    for (int k = 0; k < 3; ++k)
        if (!(p->box_hi[k] > p->box_lo[k])) return why = "box", 1;
    if (p->split_mode != APR_SPLIT_TANGENTIAL && p->split_mode != APR_SPLIT_RANDOM)
        return why = "split_mode", 1;
    return 0;
}

}  // namespace

extern "C" {

void apr_default_params(apr_params *p)
{
    std::memset(p, 0, sizeof(*p));
    p->precision = APR_FP32;
    p->kernel = APR_KERNEL_M4;
    p->eos = APR_EOS_ADIABATIC;
    p->hfact = 1.2;
    p->tol_h = 1e-6;
    p->max_iter = 50;
    p->cs0 = 1.0;
    p->q_cs = 0.25;
    p->r_ref = 1.0;
    p->gamma = 5.0 / 3.0;
    p->av_alpha = 1.0;
    p->av_beta = 2.0;
    p->periodic = 0;
    for (int k = 0; k < 3; ++k) {
        p->box_lo[k] = 0.0;
        p->box_hi[k] = 1.0;
    }
    p->m0 = 1.0;
    p->r_sep_factor = 0.2;
    p->nn_cap = 0.35;
    p->split_mode = APR_SPLIT_TANGENTIAL;
    p->ell_background = 0;
    p->derefine = 0;
    p->seed = 0;
    p->G = 1.0;
}

int apr_ctx_create(apr_ctx **out, const apr_params *p, void *stream)
{
    if (!out || !p) return APR_ERR_INVALID;
    *out = nullptr;
    std::string why;
    if (check_params(p, why)) return APR_ERR_INVALID;
    apr_ctx *c = new (std::nothrow) apr_ctx();
    if (!c) return APR_ERR_INVALID;
    c->p = *p;
    c->stream = (hipStream_t)stream;
    c->err.reserve(256);  // short messages never allocate (the allocation-free entry)
    if (hipGetDevice(&c->device) != hipSuccess ||
        hipMalloc(&c->d_status, sizeof(int32_t) * ST_WORDS) != hipSuccess ||
        hipHostMalloc(&c->h_status, sizeof(int32_t) * ST_WORDS, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc(&c->count_pin, sizeof(uint64_t), hipHostMallocCoherent) != hipSuccess ||
        hipMemsetAsync(c->d_status, 0, sizeof(int32_t) * ST_WORDS, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        if (c->d_status) (void)hipFree(c->d_status);
        if (c->h_status) (void)hipHostFree(c->h_status);
        if (c->count_pin) (void)hipHostFree(c->count_pin);
        delete c;
        return APR_ERR_HIP;
    }
    *c->count_pin = 0;  // no build has written a count yet
    if (dt_scratch_setup(c) != APR_OK) {
        (void)apr_ctx_destroy(c);
        return APR_ERR_HIP;
    }
    *out = c;
    return APR_OK;
}

int apr_ctx_destroy(apr_ctx *c)
{
    if (!c) return APR_ERR_INVALID;
    (void)hipStreamSynchronize(c->stream);
    for (auto &b : c->bufs)
        if (b.p) (void)hipFree(b.p);
    for (auto *v : {&c->ev_used, &c->ev_free})
        for (auto &e : *v) {
            (void)hipEventDestroy(e.a);
            (void)hipEventDestroy(e.b);
        }
    if (c->d_status) (void)hipFree(c->d_status);
    if (c->h_status) (void)hipHostFree(c->h_status);
    if (c->count_pin) (void)hipHostFree(c->count_pin);
    delete c;
    return APR_OK;
}

int apr_ctx_set_stream(apr_ctx *c, void *stream)
{
    if (!c) return APR_ERR_INVALID;
    c->stream = (hipStream_t)stream;
    return APR_OK;
}

int apr_set_cell_grid(apr_ctx *c, int64_t grid)
{
    if (!c) return APR_ERR_INVALID;
    if (grid < 0) return fail(c, APR_ERR_INVALID, "cell grid must be >= 0");
    c->grid_set = grid;
    return APR_OK;
}

const char *apr_last_error(const apr_ctx *c) { return c ? c->err.c_str() : "null context"; }

int apr_build_cells(apr_ctx *c, apr_state *s, int64_t *perm)
{
    int rc = check_state(c, s, false);
    if (rc) return rc;
    return build_cells(c, s, perm);
}



int apr_density(apr_ctx *c, apr_state *s, void *rho, void *omega, int32_t *nneigh,
                int32_t *iters)
{
    int rc = check_state(c, s, false);
    if (rc) return rc;
    return density(c, s, rho, omega, nneigh, iters);
}

int apr_forces(apr_ctx *c, const apr_state *s, const void *rho, const void *omega, void *ax,
               void *ay, void *az, void *dudt, void *vsig, int32_t *npair)
{
    int rc = check_state(c, s, true);
    if (rc) return rc;
    return forces(c, s, rho, omega, ax, ay, az, dudt, vsig, false, nullptr, npair);
}

int apr_vjp(apr_ctx *c, const apr_state *s, const void *rho, const void *omega,
            const void *rho_bar, const void *h_bar, const void *ax_bar, const void *ay_bar,
            const void *az_bar, const void *dudt_bar, void *xbar, void *ybar, void *zbar,
            void *mbar)
{
    int rc = check_state(c, s, true);
    if (rc) return rc;
    return vjp(c, s, rho, omega, rho_bar, h_bar, ax_bar, ay_bar, az_bar, dudt_bar, xbar, ybar,
               zbar, mbar);
}

static int check_bins(apr_ctx *c, const int8_t *bin, double dt_max, double c_cfl, int32_t max_bin,
                      const apr_sink *sinks, int32_t nsinks)
{
    if (!bin) return fail(c, APR_ERR_INVALID, "bin array required");
    if (!(dt_max > 0.0) || !(c_cfl > 0.0)) return fail(c, APR_ERR_INVALID, "dt_max, c_cfl > 0");
    if (max_bin < 0 || max_bin > 20) return fail(c, APR_ERR_INVALID, "max_bin in 0..20");
    if (nsinks < 0 || (nsinks > 0 && !sinks)) return fail(c, APR_ERR_INVALID, "sinks");
    return APR_OK;
}

int apr_bins_init(apr_ctx *c, apr_state *s, int8_t *bin, const apr_sink *sinks, int32_t nsinks,
                  double dt_max, double c_cfl, int32_t max_bin)
{
    int rc = check_state(c, s, true);
    if (rc) return rc;
    rc = check_bins(c, bin, dt_max, c_cfl, max_bin, sinks, nsinks);
    if (rc) return rc;
    if (!s->ax || !s->ay || !s->az || !s->dudt || !s->u)
        return fail(c, APR_ERR_INVALID, "state needs ax, ay, az, dudt and u");
    return bins_init(c, s, bin, sinks, nsinks, dt_max, c_cfl, max_bin);
}

int apr_step_bins(apr_ctx *c, apr_state *s, int8_t *bin, const apr_zone *zones, int32_t nzones,
                  const apr_sink *sinks, int32_t nsinks, double dt_max, double c_cfl,
                  int32_t max_bin, int64_t step, int32_t *n_substeps)
{
    int rc = check_state(c, s, true);
    if (rc) return rc;
    rc = check_bins(c, bin, dt_max, c_cfl, max_bin, sinks, nsinks);
    if (rc) return rc;
    if (!s->ax || !s->ay || !s->az || !s->dudt || !s->u)
        return fail(c, APR_ERR_INVALID, "state needs ax, ay, az, dudt and u");
    if (nzones < 0 || (nzones > 0 && !zones)) return fail(c, APR_ERR_INVALID, "zones");
    for (int k = 0; k < nzones; ++k)
        if (zones[k].n < 1 || zones[k].n > 8) return fail(c, APR_ERR_INVALID, "zone spheres");
    return step_bins(c, s, bin, zones, nzones, sinks, nsinks, dt_max, c_cfl, max_bin, step,
                     n_substeps);
}

int apr_relax(apr_ctx *c, apr_state *s, apr_ctx *rc, const apr_state *ref, const void *ref_rho,
              const void *ref_ax, const void *ref_ay, const void *ref_az, int32_t max_shuffles,
              double ke_frac, int32_t *n_shuffles, double *ke_first, double *ke_last)
{
    int r = check_state(c, s, true);
    if (r) return r;
    if (!rc || rc == c) return fail(c, APR_ERR_INVALID, "a separate reference context is needed");
    r = check_state(rc, ref, false);
    if (r) return fail(c, APR_ERR_INVALID, "reference state: " + rc->err);
    if (!ref_rho || !ref_ax || !ref_ay || !ref_az)
        return fail(c, APR_ERR_INVALID, "reference rho and accelerations are required");
    const apr_params &p = c->p, &q = rc->p;
    bool same = p.precision == q.precision && p.kernel == q.kernel && p.m0 == q.m0 &&
                p.periodic == q.periodic;
    for (int k = 0; k < 3; ++k)
        same = same && p.box_lo[k] == q.box_lo[k] && p.box_hi[k] == q.box_hi[k];
    if (!same) return fail(c, APR_ERR_INVALID, "reference context: other precision, kernel, box or m0");
    if (rc->cells_n != ref->n) return fail(c, APR_ERR_INVALID, "build the reference cells first");
    if (ref->next_id < 1 || ref->next_id > (int64_t)INT32_MAX)
        return fail(c, APR_ERR_INVALID, "reference next_id out of range");
    if (max_shuffles < 1 || max_shuffles > 1000 || !(ke_frac >= 0.0))
        return fail(c, APR_ERR_INVALID, "max_shuffles in 1..1000, ke_frac >= 0");
    if (p.eos == APR_EOS_ADIABATIC && !s->u) return fail(c, APR_ERR_INVALID, "u is required");
    return relax(c, s, rc, ref, ref_rho, ref_ax, ref_ay, ref_az, max_shuffles, ke_frac,
                 n_shuffles, ke_first, ke_last);
}

int apr_neighbours(apr_ctx *c, const apr_state *s, const double *h, int32_t mode,
                   int64_t *counts, int64_t *offsets, int64_t *list, int64_t cap,
                   int64_t *total)
{
    int rc = check_state(c, s, false);
    if (rc) return rc;
    return neighbours(c, s, h, mode, counts, offsets, list, cap, total);
}

int apr_split_merge(apr_ctx *c, apr_state *s, const apr_zone *zones, int32_t nzones,
                    int64_t step, int32_t flags, int64_t *n_split, int64_t *n_merged,
                    int64_t *n_spare)
{
    int rc = check_state(c, s, true);
    if (rc) return rc;
    if (nzones < 0 || (nzones > 0 && !zones)) return fail(c, APR_ERR_INVALID, "zones");
    for (int k = 0; k < nzones; ++k)
        if (zones[k].n < 1 || zones[k].n > 8) return fail(c, APR_ERR_INVALID, "zone spheres");
    if (!s->u) return fail(c, APR_ERR_INVALID, "state needs u");
    int64_t d0 = 0, d1 = 0, d2 = 0;
    rc = split_merge(c, s, zones, nzones, step, flags, n_split ? n_split : &d0,
                     n_merged ? n_merged : &d1, n_spare ? n_spare : &d2);
    if (rc) return rc;
    APR_HIP(c, hipStreamSynchronize(c->stream));  // the state is final on return
    return APR_OK;
}

// derived-value buffers the step and accel calls own
static void step_buffers(apr_ctx *c, int64_t cap, void **rho, void **om, void **a, void **vs)
{
    size_t e = c->p.precision == APR_FP32 ? 4 : 8;
    *rho = ws(c, "st_rho", cap * e);
    *om = ws(c, "st_om", cap * e);
    *a = ws(c, "st_acc", 4 * cap * e);
    *vs = ws(c, "st_vsig", cap * e);
}

// kick_dt != 0: the closing half-kick of a step rides on the acceleration total
static int accel_now(apr_ctx *c, apr_state *s, const apr_sink *sinks, int32_t nsinks,
                     bool build, double kick_dt = 0.0)
{
    int rc;
    if (build) {
        rc = build_cells(c, s, nullptr, false);  // accelerations recomputed below
        if (rc) return rc;
    }
    void *rho, *om, *a, *vs;
    step_buffers(c, s->capacity, &rho, &om, &a, &vs);
    if (!rho || !om || !a || !vs) return fail(c, APR_ERR_HIP, "step workspace");
    size_t e = c->p.precision == APR_FP32 ? 4 : 8;
    char *ab = (char *)a;
    size_t stride = (size_t)s->capacity * e;
    rc = density(c, s, rho, om, nullptr, nullptr);
    if (rc) return rc;
    rc = forces(c, s, rho, om, ab, ab + stride, ab + 2 * stride, ab + 3 * stride, vs, true);
    if (rc) return rc;
    return total_accel(c, s, ab, ab + stride, ab + 2 * stride, ab + 3 * stride, sinks, nsinks,
                       kick_dt);
}

int apr_accel(apr_ctx *c, apr_state *s, const apr_sink *sinks, int32_t nsinks)
{
    int rc = check_state(c, s, true);
    if (rc) return rc;
    if (!s->ax || !s->ay || !s->az || !s->dudt)
        return fail(c, APR_ERR_INVALID, "state needs ax, ay, az, dudt");
    if (nsinks > 0 && !sinks) return fail(c, APR_ERR_INVALID, "sinks");
    return accel_now(c, s, sinks, nsinks, true);
}

int apr_step(apr_ctx *c, apr_state *s, const apr_zone *zones, int32_t nzones,
             const apr_sink *sinks, int32_t nsinks, double dt, int64_t step)
{
    int rc = check_state(c, s, true);
    if (rc) return rc;
    if (!s->ax || !s->ay || !s->az || !s->dudt)
        return fail(c, APR_ERR_INVALID, "state needs ax, ay, az, dudt");
    if (nsinks > 0 && !sinks) return fail(c, APR_ERR_INVALID, "sinks");
    if (nzones < 0 || (nzones > 0 && !zones)) return fail(c, APR_ERR_INVALID, "zones");
    for (int k = 0; k < nzones; ++k)
        if (zones[k].n < 1 || zones[k].n > 8) return fail(c, APR_ERR_INVALID, "zone spheres");
    if (nzones > 0 && !s->u) return fail(c, APR_ERR_INVALID, "state needs u");
    // opening half-kick and drift, one pass; with zones the h prediction waits
    // for the refinement pass, which splits and merges with the h of the last
    // density pass
    double *hfac = nullptr;
    rc = kick_drift(c, s, 0.5 * dt, dt, nzones > 0 ? &hfac : nullptr);
    if (rc) return rc;
    if (nzones > 0) {
        // the refinement pass opens the step (before this step's density); its
        // nearest-neighbour cap uses the distances of the last density pass,
        // still in the current particle order
        int64_t ns = 0, nm = 0, nsp = 0;
        int64_t *origin = hfac ? wsa<int64_t>(c, "step_origin", (size_t)s->capacity) : nullptr;
        if (hfac && !origin) return fail(c, APR_ERR_HIP, "step workspace");
        rc = split_merge(c, s, zones, nzones, step, 0, &ns, &nm, &nsp, nullptr, origin, nullptr);
        if (rc) return rc;
        if (hfac) {
            rc = hfac_apply(c, s, origin, hfac);
            if (rc) return rc;
        }
    }
    rc = build_cells(c, s, nullptr, false);  // accelerations recomputed next
    if (rc) return rc;
    return accel_now(c, s, sinks, nsinks, false, 0.5 * dt);  // with the closing half-kick
}

int apr_timestep(apr_ctx *c, const apr_state *s, double C, double *dt)
{
    int rc = check_state(c, s, false);
    if (rc) return rc;
    if (!dt) return fail(c, APR_ERR_INVALID, "dt");
    if (c->force_n != s->n) return fail(c, APR_ERR_INVALID, "no force evaluation for this state");
    void *rho, *om, *a, *vs;
    step_buffers(c, s->capacity, &rho, &om, &a, &vs);
    return min_timestep(c, s, vs, C, dt);
}

int apr_timestep_noalloc(apr_ctx *c, const apr_state *s, double C, double *dt_dev)
{
    int rc = check_state(c, s, false);
    if (rc) return rc;
    if (!dt_dev) return fail(c, APR_ERR_INVALID, "dt_dev");
    if (c->force_n != s->n) return fail(c, APR_ERR_INVALID, "no force evaluation for this state");
    const size_t e = c->p.precision == APR_FP32 ? 4 : 8;
    const void *vs = ws_peek(c, "st_vsig", (size_t)s->capacity * e);
    if (!vs) return fail(c, APR_ERR_INVALID, "no force evaluation for this state");
    return min_timestep_noalloc(c, s, vs, C, dt_dev);
}

int apr_profile_enable(apr_ctx *c, int on)
{
    if (!c) return APR_ERR_INVALID;
    c->prof = on != 0;
    return APR_OK;
}

int apr_profile_select(apr_ctx *c, uint32_t mask)
{
    if (!c) return APR_ERR_INVALID;
    c->prof_mask = mask;
    return APR_OK;
}

int apr_profile_read(apr_ctx *c, double *ms, int64_t *launches, int reset)
{
    if (!c) return APR_ERR_INVALID;
    APR_HIP(c, hipStreamSynchronize(c->stream));
    for (auto &e : c->ev_used) {
        float t = 0.0f;
        APR_HIP(c, hipEventElapsedTime(&t, e.a, e.b));
        c->prof_ms[e.idx] += t;
        c->prof_cnt[e.idx] += 1;
        c->ev_free.push_back(e);
    }
    c->ev_used.clear();
    for (int k = 0; k < APR_PROF_N; ++k) {
        if (ms) ms[k] = c->prof_ms[k];
        if (launches) launches[k] = c->prof_cnt[k];
        if (reset) {
            c->prof_ms[k] = 0.0;
            c->prof_cnt[k] = 0;
        }
    }
    return APR_OK;
}

int apr_counters(apr_ctx *c, int64_t *out, int reset)
{
    if (!c || !out) return APR_ERR_INVALID;
    APR_HIP(c, hipMemcpyAsync(c->h_status, c->d_status, sizeof(int32_t) * ST_WORDS,
                              hipMemcpyDeviceToHost, c->stream));
    APR_HIP(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < APR_COUNTERS_N; ++k) out[k] = k < ST_WORDS ? c->h_status[k] : 0;
    if (reset) {
        int rc = fill_i32(c, c->d_status, 0, ST_WORDS);
        if (rc) return rc;
        APR_HIP(c, hipStreamSynchronize(c->stream));
    }
    return APR_OK;
}

int apr_sync_status(apr_ctx *c, int64_t *count)
{
    if (!c) return APR_ERR_INVALID;
    APR_HIP(c, hipMemcpyAsync(c->h_status, c->d_status, sizeof(int32_t) * ST_WORDS,
                              hipMemcpyDeviceToHost, c->stream));
    APR_HIP(c, hipStreamSynchronize(c->stream));
    // the flags are cleared; the work counters [ST_DENS_DIRECT..] are kept
    APR_HIP(c, hipMemsetAsync(c->d_status, 0, sizeof(int32_t) * 2, c->stream));
    int32_t nc = c->h_status[ST_NOCONV], ov = c->h_status[ST_RANGE];
    if (count) *count = nc;
    if (ov)
        return fail(c, APR_ERR_RANGE,
                    "a smoothing length reached the periodic limit (2 h < a quarter of the box)");
    if (nc) return fail(c, APR_ERR_NOCONVERGE, std::to_string(nc) + " h-rho solves did not converge");
    return APR_OK;
}

}  // extern "C"
