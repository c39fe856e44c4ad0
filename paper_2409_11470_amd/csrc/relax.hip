// Relaxing after a split/merge pass (paper Sec. 2.4).  The particles the pass
// introduced (new ids, or a level that differs from the reference set's for
// the same id) are shuffled, repeatedly:
//   a_new   hydro accelerations of the new set at its current positions
//           (cells, density with its h-rho solve, forces: the path's kernels);
//   a_ref   the reference set's accelerations at the same points, by the
//           reference set's own SPH interpolant
//             a_ref(x) = sum_b (m_b / rho_b) a_b W(|x - x_b|, h_b)
//           over r < 2 h_b (a walk of the reference set's cell tree);
//   dx      0.5 dt^2 (a_new - a_ref) with dt = 0.3 h / c_s of the particle,
//           its length capped at h;
//   KE      sum |dx| / dt^2 over the shuffled particles,
// until KE has fallen to ke_frac of the first shuffle's, or max shuffles.
// The interpolation and the shift are FP64 whatever the form; KE is summed
// in a fixed order (per-block partials, then one block), so the stopping
// decision is reproducible.
#include "search.hpp"
#include "sph_kernel.hpp"

namespace apr {

Tree make_tree(apr_ctx *c, const apr_state *s);

namespace {

constexpr int kRelaxThreads = 256;
constexpr int kKeBlocks = 1024;

__global__ void k_fill_i8(int8_t *p, int8_t v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// level of every reference particle by id (ids are below the reference's next_id)
__global__ void k_ref_levels(int64_t n, const int64_t *id, const int8_t *level, int64_t nid,
                             int8_t *tbl)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t k = id[i];
    if (k >= 0 && k < nid) tbl[k] = level[i];
}

// q_b = (m_b / rho_b) a_b of every reference particle, FP64
template <class T>
__global__ void k_ref_pack(int64_t n, const int8_t *level, double m0, const T *rho, const T *ax,
                           const T *ay, const T *az, double *q0, double *q1, double *q2)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double w = ldexp(m0, -(int)level[i]) / (double)rho[i];
    q0[i] = w * (double)ax[i];
    q1[i] = w * (double)ay[i];
    q2[i] = w * (double)az[i];
}

struct InterpArgs {
    Tree src, tgt;                  // reference set's cells, new set's cells
    const double *x, *y, *z;        // new set (its cell order)
    const double *rx, *ry, *rz, *rh; // reference set (its cell order)
    const double *q0, *q1, *q2;
    double *o0, *o1, *o2;           // a_ref of the new set
    Box box;
};

__device__ inline double min_image(double d, const Box &b, int k)
{
    if (b.periodic) {
        if (d > 0.5 * b.L[k]) d -= b.L[k];
        else if (d < -0.5 * b.L[k]) d += b.L[k];
    }
    return d;
}

// One workgroup per cell of the new set: the reference cells whose
// particles can reach the cell (walk with radius 2 h_max of each node),
// then 4 lanes per target over their particles, summed in a fixed order.
template <int K>
__global__ __launch_bounds__(kRelaxThreads) void k_interp(InterpArgs a)
{
    __shared__ int32_t sA[kCandCap];
    __shared__ Walk s_walk;
    __shared__ int s_nc, s_more;
    const int64_t nct = a.tgt.hdr->ncells;
    const int w = threadIdx.x / kWave, lane = lane_id();
    const int t = threadIdx.x >> 2, j = threadIdx.x & 3;
    for (int64_t cell = blockIdx.x; cell < nct; cell += gridDim.x) {
        const Geo tg = a.tgt.lev[0][cell];
        const int32_t s0 = a.tgt.cs[cell];
        const int cnt = a.tgt.cs[cell + 1] - s0;
        const bool valid = t < cnt;
        const double px = valid ? a.x[s0 + t] : 0.0, py = valid ? a.y[s0 + t] : 0.0,
                     pz = valid ? a.z[s0 + t] : 0.0;
        double s[3] = {0.0, 0.0, 0.0};
        __syncthreads();  // the previous cell's walk state is no longer read
        if (w == 0) walk_init(a.src, tg, 0.0, true, &s_walk);
        for (;;) {
            __syncthreads();
            if (w == 0) {
                int k = walk_next(a.src, tg, 0.0, true, &s_walk, sA, kCandCap);
                if (lane == 0) {
                    s_nc = k;
                    s_more = walk_done(a.src, &s_walk) ? 0 : 1;
                }
            }
            __syncthreads();
            const int nc = s_nc;
            const bool more = s_more != 0;
            if (valid) {
                for (int ci = 0; ci < nc; ++ci) {
                    const int32_t c = sA[ci];
                    const int32_t b1 = a.src.cs[c + 1];
                    for (int32_t b = a.src.cs[c] + j; b < b1; b += 4) {
                        double dx = min_image(px - a.rx[b], a.box, 0);
                        double dy = min_image(py - a.ry[b], a.box, 1);
                        double dz = min_image(pz - a.rz[b], a.box, 2);
                        double r2 = dx * dx + dy * dy + dz * dz;
                        double hb = a.rh[b];
                        double R = 2.0 * hb;
                        if (!(r2 < R * R)) continue;
                        double f, df, d2f;
                        Kern<K>::template eval<double, 0>(sqrt(r2) / hb, f, df, d2f);
                        double wgt = f / (hb * hb * hb);
                        s[0] += a.q0[b] * wgt;
                        s[1] += a.q1[b] * wgt;
                        s[2] += a.q2[b] * wgt;
                    }
                }
            }
            if (!more) break;
        }
        // the target's 4 lanes, in lane order
        for (int k = 0; k < 3; ++k) {
            double v0 = __shfl(s[k], (lane & ~3) + 0, kWave);
            double v1 = __shfl(s[k], (lane & ~3) + 1, kWave);
            double v2 = __shfl(s[k], (lane & ~3) + 2, kWave);
            double v3 = __shfl(s[k], (lane & ~3) + 3, kWave);
            s[k] = ((v0 + v1) + v2) + v3;
        }
        if (valid && j == 0) {
            const double ip = 1.0 / kPi;
            a.o0[s0 + t] = s[0] * ip;
            a.o1[s0 + t] = s[1] * ip;
            a.o2[s0 + t] = s[2] * ip;
        }
    }
}

struct ShiftArgs {
    int64_t n;
    double *x, *y, *z;
    const double *h;
    const int8_t *level;
    const int64_t *id;
    const int8_t *tbl;  // reference level by id
    int64_t ref_next_id;
    const double *ar0, *ar1, *ar2;
    Box box;
    double *partial;    // per block: sum of |dx| / dt^2
};

// The shift of every introduced particle; per-block KE partials.
template <class T>
__global__ __launch_bounds__(kRelaxThreads) void k_relax_shift(ShiftArgs a, const T *ax,
                                                               const T *ay, const T *az,
                                                               const vec4_t<T> *th)
{
    __shared__ double red[kRelaxThreads / kWave];
    double ke = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t id = a.id[i];
        const bool introduced = id >= a.ref_next_id || id < 0 || a.tbl[id] != a.level[i];
        if (!introduced) continue;
        const double h = a.h[i];
        const double dt = 0.3 * h / (double)th[i].z;
        const double c = 0.5 * dt * dt;
        double d[3] = {c * ((double)ax[i] - a.ar0[i]), c * ((double)ay[i] - a.ar1[i]),
                       c * ((double)az[i] - a.ar2[i])};
        double ln = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (ln > h) {
            const double sc = h / ln;
            for (int k = 0; k < 3; ++k) d[k] *= sc;
            ln = h;
        }
        double *p[3] = {a.x, a.y, a.z};
        for (int k = 0; k < 3; ++k) {
            double v = p[k][i] + d[k];
            if (a.box.periodic) {  // one image back into [lo, lo + L)
                const double hi = a.box.lo[k] + a.box.L[k];
                if (v >= hi) v -= a.box.L[k];
                else if (v < a.box.lo[k]) v += a.box.L[k];
            }
            p[k][i] = v;
        }
        ke += ln / (dt * dt);
    }
    // fixed-order reduction: wavefront tree, then the wavefronts in order
    for (int o = kWave / 2; o > 0; o >>= 1) ke += __shfl_down(ke, o, kWave);
    if (lane_id() == 0) red[threadIdx.x / kWave] = ke;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < kRelaxThreads / kWave; ++k) s += red[k];
        a.partial[blockIdx.x] = s;
    }
}

__global__ void k_sum_partials(const double *partial, int nb, double *out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < nb; ++k) s += partial[k];
        *out = s;
    }
}

}  // namespace

int relax(apr_ctx *c, apr_state *s, apr_ctx *rc, const apr_state *ref, const void *ref_rho,
          const void *ref_ax, const void *ref_ay, const void *ref_az, int32_t max_shuffles,
          double ke_frac, int32_t *n_shuffles, double *ke_first, double *ke_last)
{
    const apr_params &P = c->p;
    const int64_t nr = ref->n, nid = ref->next_id;
    const bool f32 = P.precision == APR_FP32;
    // the reference set: levels by id, and q_b = (m_b / rho_b) a_b
    int8_t *tbl = wsa<int8_t>(c, "rx_tbl", (size_t)nid);
    double *q[3] = {wsa<double>(c, "rx_q0", (size_t)nr), wsa<double>(c, "rx_q1", (size_t)nr),
                    wsa<double>(c, "rx_q2", (size_t)nr)};
    double *partial = wsa<double>(c, "rx_part", (size_t)kKeBlocks);
    double *ke_dev = wsa<double>(c, "rx_ke", 1);
    if (!tbl || !q[0] || !q[1] || !q[2] || !partial || !ke_dev)
        return fail(c, APR_ERR_HIP, "relax workspace");
    hipLaunchKernelGGL(k_fill_i8, dim3((unsigned)ceil_div(nid, 256)), dim3(256), 0, c->stream,
                       tbl, (int8_t)-1, nid);
    hipLaunchKernelGGL(k_ref_levels, dim3((unsigned)ceil_div(nr, 256)), dim3(256), 0, c->stream,
                       nr, ref->id, ref->level, nid, tbl);
    if (f32)
        hipLaunchKernelGGL(k_ref_pack<float>, dim3((unsigned)ceil_div(nr, 256)), dim3(256), 0,
                           c->stream, nr, ref->level, P.m0, (const float *)ref_rho,
                           (const float *)ref_ax, (const float *)ref_ay, (const float *)ref_az,
                           q[0], q[1], q[2]);
    else
        hipLaunchKernelGGL(k_ref_pack<double>, dim3((unsigned)ceil_div(nr, 256)), dim3(256), 0,
                           c->stream, nr, ref->level, P.m0, (const double *)ref_rho,
                           (const double *)ref_ax, (const double *)ref_ay,
                           (const double *)ref_az, q[0], q[1], q[2]);
    APR_LAUNCHED(c);
    // the reference set's work must be done before its stream's results are read
    if (rc->stream != c->stream) APR_HIP(c, hipStreamSynchronize(rc->stream));

    double ke0 = 0.0, ke = 0.0;
    int k = 0;
    while (k < max_shuffles) {
        const int64_t n = s->n;
        int r = build_cells(c, s, nullptr, false);
        if (r) return r;
        void *rho = ws(c, "rx_rho", (size_t)n * 8 + 256), *om = ws(c, "rx_om", (size_t)n * 8 + 256);
        void *an[4] = {ws(c, "rx_ax", (size_t)n * 8 + 256), ws(c, "rx_ay", (size_t)n * 8 + 256),
                       ws(c, "rx_az", (size_t)n * 8 + 256), ws(c, "rx_du", (size_t)n * 8 + 256)};
        double *ar[3] = {wsa<double>(c, "rx_ar0", (size_t)n), wsa<double>(c, "rx_ar1", (size_t)n),
                         wsa<double>(c, "rx_ar2", (size_t)n)};
        if (!rho || !om || !an[0] || !an[1] || !an[2] || !an[3] || !ar[0] || !ar[1] || !ar[2])
            return fail(c, APR_ERR_HIP, "relax workspace");
        r = density(c, s, rho, om, nullptr, nullptr);
        if (r) return r;
        r = forces(c, s, rho, om, an[0], an[1], an[2], an[3], nullptr);
        if (r) return r;
        InterpArgs ia;
        ia.src = make_tree(rc, ref);
        ia.tgt = make_tree(c, s);
        ia.x = s->x;
        ia.y = s->y;
        ia.z = s->z;
        ia.rx = ref->x;
        ia.ry = ref->y;
        ia.rz = ref->z;
        ia.rh = ref->h;
        ia.q0 = q[0];
        ia.q1 = q[1];
        ia.q2 = q[2];
        ia.o0 = ar[0];
        ia.o1 = ar[1];
        ia.o2 = ar[2];
        ia.box = make_box(P);
        const unsigned gi = (unsigned)std::max<int64_t>(1, c->node_grid[0]);
        if (P.kernel == APR_KERNEL_WC2)
            hipLaunchKernelGGL(k_interp<kWC2>, dim3(gi), dim3(kRelaxThreads), 0, c->stream, ia);
        else
            hipLaunchKernelGGL(k_interp<kM4>, dim3(gi), dim3(kRelaxThreads), 0, c->stream, ia);
        ShiftArgs sa;
        sa.n = n;
        sa.x = s->x;
        sa.y = s->y;
        sa.z = s->z;
        sa.h = s->h;
        sa.level = s->level;
        sa.id = s->id;
        sa.tbl = tbl;
        sa.ref_next_id = nid;
        sa.ar0 = ar[0];
        sa.ar1 = ar[1];
        sa.ar2 = ar[2];
        sa.box = ia.box;
        sa.partial = partial;
        const int nb = (int)std::min<int64_t>(kKeBlocks, ceil_div(n, kRelaxThreads));
        if (f32)
            hipLaunchKernelGGL(k_relax_shift<float>, dim3(nb), dim3(kRelaxThreads), 0, c->stream,
                               sa, (const float *)an[0], (const float *)an[1],
                               (const float *)an[2], wsa<float4>(c, "th32", (size_t)n));
        else
            hipLaunchKernelGGL(k_relax_shift<double>, dim3(nb), dim3(kRelaxThreads), 0,
                               c->stream, sa, (const double *)an[0], (const double *)an[1],
                               (const double *)an[2], wsa<double4>(c, "th64", (size_t)n));
        hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, c->stream, partial, nb, ke_dev);
        APR_LAUNCHED(c);
        APR_HIP(c, hipMemcpyAsync(&ke, ke_dev, 8, hipMemcpyDeviceToHost, c->stream));
        APR_HIP(c, hipStreamSynchronize(c->stream));
        // positions moved: the cells and everything derived from them are stale
        c->cells_n = -1;
        c->dens_n = -1;
        c->force_n = -1;
        c->divv_n = -1;
        c->divv_prev_n = -1;
        if (k == 0) ke0 = ke;
        ++k;
        if (ke <= ke_frac * ke0) break;
    }
    if (n_shuffles) *n_shuffles = k;
    if (ke_first) *ke_first = ke0;
    if (ke_last) *ke_last = ke;
    return APR_OK;
}

}  // namespace apr
