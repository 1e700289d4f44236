// ebic_batch.cpp -- ebic_eval_batch: many populations in one call.
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/ebic.h"
#include "ebic_internal.h"
#include "ebic_runtime_internal.h"

namespace ebic {

struct BatchState {};

void destroy_batch_state(ebic_ctx *ctx)
{
    delete ctx->batch;
    ctx->batch = nullptr;
    ctx->batch_state_allocated = false;
}

}  // namespace ebic

using namespace ebic;

extern "C" ebic_status ebic_eval_batch(ebic_ctx *ctx, const ebic_request *reqs, int32_t n_reqs,
                                       void *hip_stream)
{
    if (!ctx || n_reqs < 0 || (n_reqs > 0 && !reqs)) return EBIC_EINVAL;
    for (int32_t q = 0; q < n_reqs; ++q) {
        const ebic_request &r = reqs[q];
        ebic_status st = ebic_eval_population(ctx, r.matrix, r.n_ind, r.d_offsets, r.d_cols, r.flags,
                                              r.d_matched, r.d_negative, r.d_matched_mask,
                                              r.d_negative_mask, hip_stream);
        if (st != EBIC_OK) return st;
    }
    return EBIC_OK;
}
