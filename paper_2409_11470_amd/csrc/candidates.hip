// Candidate cells of every leaf cell, found ahead of the search kernels: one
// wavefront per cell walks the tree (so that many walks are in flight at
// once, instead of one wavefront of a 4-wavefront workgroup walking while the
// other three wait).  The search kernels load the list with one coalesced
// read.  A cell whose walk needs more than one chunk gets -1 and its search
// kernel walks by itself.
#include "search.hpp"

namespace apr {

namespace {

static_assert(kCell <= kWave, "one lane per target of a cell");

// act (optional): a cell none of whose targets is active gets an empty list
// and no walk (the search kernels leave such a cell before reading it)
template <bool SYM>
__global__ __launch_bounds__(kWave) void k_cand_pre(Tree tr, double rfac, const uint8_t *act,
                                                    int32_t *cand, int32_t *ncand, int64_t cap)
{
    __shared__ int32_t A[kCandCap];
    __shared__ Walk W;
    const int lane = lane_id();
    const int64_t nc = min((int64_t)tr.hdr->ncells, cap);
    for (int64_t cell = first_cell(blockIdx.x, gridDim.x, nc); cell >= 0 && cell < nc;
         cell += gridDim.x) {
        if (act) {
            const int32_t s0 = tr.cs[cell];
            const int cnt = tr.cs[cell + 1] - s0;  // at most kCell = one lane per target
            if (!__any(lane < cnt && act[s0 + lane] != 0)) {
                if (lane == 0) ncand[cell] = 0;
                continue;
            }
        }
        const Geo tg = tr.lev[0][cell];
        const double R = rfac * (double)tg.hmax;
        walk_init(tr, tg, R, SYM, &W);
        int n = walk_next(tr, tg, R, SYM, &W, A, kCandCap);
        bool done = walk_done(tr, &W);
        for (int k = lane; k < n; k += kWave) cand[cell * kCandCap + k] = A[k];
        if (lane == 0) ncand[cell] = done ? n : -1;
        wave_sync();  // A and W are rewritten for the next cell
    }
}

}  // namespace

int cand_pre(apr_ctx *c, const Tree &tr, bool sym, double rfac, CandList *out,
             const uint8_t *active)
{
    // lists for the cells the host expects (the launch grid of the search
    // kernels); any cells beyond walk in the search kernel
    const int64_t grid = c->node_grid[0], cap = std::min(c->node_cap[0], grid);
    int32_t *cand = wsa<int32_t>(c, sym ? "cand_sym" : "cand_gat", (size_t)cap * kCandCap);
    int32_t *ncand = wsa<int32_t>(c, sym ? "ncand_sym" : "ncand_gat", (size_t)cap);
    if (!cand || !ncand) return fail(c, APR_ERR_HIP, "candidate workspace");
    int tok = prof_begin(c, APR_PROF_CAND);
    if (sym)
        hipLaunchKernelGGL(k_cand_pre<true>, dim3((unsigned)grid), dim3(kWave), 0, c->stream, tr,
                           rfac, active, cand, ncand, cap);
    else
        hipLaunchKernelGGL(k_cand_pre<false>, dim3((unsigned)grid), dim3(kWave), 0, c->stream,
                           tr, rfac, active, cand, ncand, cap);
    prof_end(c, tok);
    APR_LAUNCHED(c);
    out->cand = cand;
    out->ncand = ncand;
    out->rfac = rfac;
    out->cap = cap;
    return APR_OK;
}

}  // namespace apr
