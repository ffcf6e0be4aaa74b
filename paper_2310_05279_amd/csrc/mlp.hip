// Learned C6 surrogate (placeholder until the training and inference
// kernels land): every entry point reports D3_ERR_NOT_TRAINED.
#include "d3_ctx.h"

namespace d3 {
void surrogate_free(d3_ctx* c)
{
    if (c && c->sur) {
        delete c->sur;
        c->sur = nullptr;
    }
}
int surrogate_pair(d3_ctx*, const PairScal&, hipStream_t)
{
    return fail(D3_ERR_NOT_TRAINED, "surrogate not available");
}
}  // namespace d3

using namespace d3;
extern "C" {
int d3_c6_surrogate_init(d3_ctx*, uint64_t) { return fail(D3_ERR_NOT_TRAINED, "not available"); }
int d3_c6_surrogate_train(d3_ctx*, const d3_train_cfg*, double*, void*) { return fail(D3_ERR_NOT_TRAINED, "not available"); }
int d3_c6_surrogate_eval(d3_ctx*, int64_t, const int32_t*, const int32_t*, const float*, const float*, float*, int32_t, void*) { return fail(D3_ERR_NOT_TRAINED, "not available"); }
int d3_c6_exact_eval(d3_ctx*, int64_t, const int32_t*, const int32_t*, const double*, const double*, double*, void*) { return fail(D3_ERR_NOT_TRAINED, "not available"); }
int64_t d3_c6_surrogate_bytes(d3_ctx*) { return 0; }
int d3_c6_surrogate_get_weights(d3_ctx*, float*, int64_t) { return fail(D3_ERR_NOT_TRAINED, "not available"); }
int d3_c6_surrogate_set_weights(d3_ctx*, const float*, int64_t) { return fail(D3_ERR_NOT_TRAINED, "not available"); }
int d3_c6_surrogate_grad(d3_ctx*, int64_t, const int32_t*, const float*, const float*, float*, float*, void*) { return fail(D3_ERR_NOT_TRAINED, "not available"); }
int d3_md_nve(d3_ctx*, int64_t, double, double*, double*, const double*, int32_t, double*, int64_t*, void*) { return fail(D3_ERR_STATE, "not available"); }
}
