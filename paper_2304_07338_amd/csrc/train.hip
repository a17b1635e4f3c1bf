// Field training (Section 3.5): batch generation, fused forward/backward, Adam.
#include "pfn_ctx.h"

extern "C" pfn_status pfn_train_field(pfn_context *ctx, const pfn_train_params *, float *) {
  if (!ctx) return PFN_ERR_INVALID_ARG;
  return pfn_fail(ctx, PFN_ERR_UNSUPPORTED, "training not built yet");
}
extern "C" pfn_status pfn_train_batch(pfn_context *ctx, uint64_t, int64_t, int64_t, float *, float *,
                                      float *, int32_t *, float *) {
  if (!ctx) return PFN_ERR_INVALID_ARG;
  return pfn_fail(ctx, PFN_ERR_UNSUPPORTED, "training not built yet");
}
extern "C" pfn_status pfn_field_forward_backward(pfn_context *ctx, pfn_dtype, const float *,
                                                 const float *, const float *, const float *,
                                                 int64_t, double *, float *) {
  if (!ctx) return PFN_ERR_INVALID_ARG;
  return pfn_fail(ctx, PFN_ERR_UNSUPPORTED, "training not built yet");
}
extern "C" pfn_status pfn_field_adam_step(pfn_context *ctx, const float *, int64_t, float, float,
                                          float, float) {
  if (!ctx) return PFN_ERR_INVALID_ARG;
  return pfn_fail(ctx, PFN_ERR_UNSUPPORTED, "training not built yet");
}
