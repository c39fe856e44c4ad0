// Neighbour-list export with the exact FP64 predicate (test interface):
//   mode 0: b != a with r_ab^2 < (2 h_a)^2
//   mode 1: b != a with r_ab^2 < (2 h_a)^2 or r_ab^2 < (2 h_b)^2
// on absolute positions, minimum image, dx*dx + dy*dy + dz*dz summed left to
// right with every product and sum rounded on its own (no contraction), so
// that membership is decided bit for bit like a plain FP64 evaluation.
#include "search.hpp"

namespace apr {

Tree make_tree(apr_ctx *c, const apr_state *s);

namespace {

__device__ inline double sep_exact(double a, double b, double L, int periodic)
{
#pragma clang fp contract(off)
    double d = a - b;
    if (periodic) {
        if (d > 0.5 * L) d -= L;
        else if (d < -0.5 * L) d += L;
    }
    return d;
}

__device__ inline bool is_neighbour(double xa, double ya, double za, double ha, double xb,
                                    double yb, double zb, double hb, const Box &b, int mode)
{
#pragma clang fp contract(off)
    double dx = sep_exact(xa, xb, b.L[0], b.periodic);
    double dy = sep_exact(ya, yb, b.L[1], b.periodic);
    double dz = sep_exact(za, zb, b.L[2], b.periodic);
    double r2 = dx * dx + dy * dy + dz * dz;
    double Ra = 2.0 * ha, Rb = 2.0 * hb;
    bool in = r2 < Ra * Ra;
    if (mode == 1 && !in) in = r2 < Rb * Rb;
    return in;
}

// one wavefront per target cell (striding over the device's cell count);
// lane = target
__global__ __launch_bounds__(64) void k_neigh(Tree tr, const double *x, const double *y,
                                              const double *z, const double *h, int mode,
                                              int64_t *counts, const int64_t *offsets,
                                              int64_t *list, int64_t cap)
{
    __shared__ int32_t sA[kCandCap];
    __shared__ Walk s_walk;
    const int lane = lane_id();
    const int64_t ncells = tr.hdr->ncells;
    for (int64_t cell = first_cell(blockIdx.x, gridDim.x, ncells); cell >= 0 && cell < ncells;
         cell += gridDim.x) {
        const Geo tg = tr.lev[0][cell];
        int32_t s0 = tr.cs[cell], s1 = tr.cs[cell + 1];
        int64_t a = s0 + lane;
        bool valid = a < s1;
        double xa = valid ? x[a] : 0.0, ya = valid ? y[a] : 0.0, za = valid ? z[a] : 0.0;
        double ha = valid ? h[a] : 0.0;
        int64_t k = 0;
        int64_t off = (list && valid) ? offsets[a] : 0;
        const double R = 2.0 * (double)tg.hmax;
        walk_init(tr, tg, R, mode == 1, &s_walk);
        for (;;) {
            int nc = walk_next(tr, tg, R, mode == 1, &s_walk, sA, kCandCap);
            for (int ci = 0; ci < nc; ++ci) {
                int cc = sA[ci];
                int32_t b0 = tr.cs[cc], b1 = tr.cs[cc + 1];
                for (int32_t b = b0; b < b1; ++b) {
                    double xb = x[b], yb = y[b], zb = z[b], hb = h[b];
                    if (valid && b != a &&
                        is_neighbour(xa, ya, za, ha, xb, yb, zb, hb, tr.box, mode)) {
                        if (list && off + k < cap) list[off + k] = b;
                        k += 1;
                    }
                }
            }
            wave_sync();  // sA is read before the next chunk is written
            if (walk_done(tr, &s_walk)) break;
        }
        if (valid && !list) counts[a] = k;
        wave_sync();  // the walk state is rewritten for the next cell
    }
}

}  // namespace

int neighbours(apr_ctx *c, const apr_state *s, const double *h, int mode, int64_t *counts,
               int64_t *offsets, int64_t *list, int64_t cap, int64_t *total)
{
    if (c->cells_n != s->n) return fail(c, APR_ERR_INVALID, "apr_build_cells first");
    if (mode != 0 && mode != 1) return fail(c, APR_ERR_INVALID, "mode must be 0 or 1");
    if (!h || !counts || !offsets) return fail(c, APR_ERR_INVALID, "null argument");
    int64_t n = s->n;
    int rc = cells_hmax_from(c, h, n);
    if (rc) return rc;
    Tree tr = make_tree(c, s);
    unsigned nb = (unsigned)c->node_grid[0];
    if (!list) {
        hipLaunchKernelGGL(k_neigh, dim3(nb), dim3(64), 0, c->stream, tr, s->x, s->y, s->z, h,
                           mode, counts, offsets, (int64_t *)nullptr, (int64_t)0);
        APR_LAUNCHED(c);
        int64_t *tot = wsa<int64_t>(c, "neigh_total", 1);
        rc = exclusive_scan_i64(c, counts, offsets, n, tot);
        if (rc) return rc;
        APR_HIP(c, hipMemcpyAsync(offsets + n, tot, sizeof(int64_t), hipMemcpyDeviceToDevice,
                                  c->stream));
        int64_t t = 0;
        APR_HIP(c, hipMemcpyAsync(&t, tot, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
        APR_HIP(c, hipStreamSynchronize(c->stream));
        if (total) *total = t;
        return APR_OK;
    }
    hipLaunchKernelGGL(k_neigh, dim3(nb), dim3(64), 0, c->stream, tr, s->x, s->y, s->z, h, mode,
                       counts, offsets, list, cap);
    APR_LAUNCHED(c);
    return APR_OK;
}

}  // namespace apr
