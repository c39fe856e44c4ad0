// Split/merge pass (placeholder until the GPU pass lands).
#include "common.hpp"

namespace apr {

int split_merge(apr_ctx *c, apr_state *, const apr_zone *, int, int64_t, int, int64_t *,
                int64_t *, int64_t *)
{
    return fail(c, APR_ERR_INVALID, "split/merge pass not available in this build");
}

}  // namespace apr
