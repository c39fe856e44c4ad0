// Candidate cells of every leaf cell, found ahead of the search kernels: one
// wavefront per cell walks the tree (so that many walks are in flight at
// once, instead of one wavefront of a 4-wavefront workgroup walking while the
// other three wait).  The search kernels load the list with one coalesced
// read.  A cell whose walk needs more than one chunk gets -1 and its search
// kernel walks by itself.
#include "search.hpp"

namespace apr {

namespace {

template <bool SYM>
__global__ __launch_bounds__(kWave) void k_cand_pre(Tree tr, double rfac, int32_t *cand,
                                                    int32_t *ncand)
{
    __shared__ int32_t A[kCandCap];
    __shared__ Walk W;
    int64_t cell = xcd_swizzle(blockIdx.x, gridDim.x);
    if (cell >= tr.hdr->ncells) return;
    const Geo tg = tr.lev[0][cell];
    const double R = rfac * (double)tg.hmax;
    walk_init(tr, tg, R, SYM, &W);
    int n = walk_next(tr, tg, R, SYM, &W, A, kCandCap);
    bool done = walk_done(tr, &W);
    int lane = lane_id();
    for (int k = lane; k < n; k += kWave) cand[cell * kCandCap + k] = A[k];
    if (lane == 0) ncand[cell] = done ? n : -1;
}

}  // namespace

int cand_pre(apr_ctx *c, const Tree &tr, bool sym, double rfac, CandList *out)
{
    int64_t cb = c->cells_bound;
    int32_t *cand = wsa<int32_t>(c, sym ? "cand_sym" : "cand_gat", (size_t)cb * kCandCap);
    int32_t *ncand = wsa<int32_t>(c, sym ? "ncand_sym" : "ncand_gat", (size_t)cb);
    if (!cand || !ncand) return fail(c, APR_ERR_HIP, "candidate workspace");
    int tok = prof_begin(c, APR_PROF_CAND);
    if (sym)
        hipLaunchKernelGGL(k_cand_pre<true>, dim3((unsigned)cb), dim3(kWave), 0, c->stream, tr,
                           rfac, cand, ncand);
    else
        hipLaunchKernelGGL(k_cand_pre<false>, dim3((unsigned)cb), dim3(kWave), 0, c->stream, tr,
                           rfac, cand, ncand);
    prof_end(c, tok);
    APR_LAUNCHED(c);
    out->cand = cand;
    out->ncand = ncand;
    out->rfac = rfac;
    return APR_OK;
}

}  // namespace apr
