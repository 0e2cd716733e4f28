// stubs.hip -- entry points whose full implementation lives elsewhere.
#include "abi_internal.h"
struct SizerState {};
struct BatchState {};
void sizer_init(aiwc_ctx *) {}
void sizer_free(aiwc_ctx *) {}
void batch_free(aiwc_ctx *) {}

#define UNSUP(ctx)                                                      \
  do { ctx_error(ctx, "not implemented in this build"); return AIWC_ERR_UNSUPPORTED; } while (0)

extern "C" {
aiwc_status aiwc_characterize_batch(aiwc_ctx *ctx, const aiwc_trace *const *, size_t,
                                    const aiwc_batch_opts *, void *, aiwc_metrics **) { UNSUP(ctx); }
aiwc_status aiwc_batch_last_stats(const aiwc_ctx *ctx, aiwc_batch_stats *) { UNSUP((aiwc_ctx *)ctx); }
aiwc_status aiwc_sizer_features(aiwc_ctx *ctx, const aiwc_trace *const *, size_t, void *, float *) { UNSUP(ctx); }
aiwc_status aiwc_sizer_train(aiwc_ctx *ctx, const float *, const float *, size_t,
                             const aiwc_train_opts *, void *, float *) { UNSUP(ctx); }
aiwc_status aiwc_sizer_predict(aiwc_ctx *ctx, const float *, size_t, void *, float *) { UNSUP(ctx); }
aiwc_status aiwc_sizer_grad(aiwc_ctx *ctx, const float *, const float *, size_t, void *, float *,
                            float *) { UNSUP(ctx); }
size_t aiwc_sizer_num_params(void) { return 0; }
aiwc_status aiwc_sizer_get_params(const aiwc_ctx *ctx, float *) { UNSUP((aiwc_ctx *)ctx); }
aiwc_status aiwc_sizer_set_params(aiwc_ctx *ctx, const float *) { UNSUP(ctx); }
aiwc_status aiwc_sizer_save(const aiwc_ctx *ctx, const char *) { UNSUP((aiwc_ctx *)ctx); }
aiwc_status aiwc_sizer_load(aiwc_ctx *ctx, const char *) { UNSUP(ctx); }
aiwc_status aiwc_sizer_set_margin(aiwc_ctx *ctx, float) { UNSUP(ctx); }
}
