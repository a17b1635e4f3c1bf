// Monte Carlo volumetric path tracer and image error metrics.
#include "pfn_ctx.h"

extern "C" pfn_status pfn_render_path_traced(pfn_context *ctx, const pfn_camera *, int, int, float,
                                             int, int, uint64_t, float *) {
  if (!ctx) return PFN_ERR_INVALID_ARG;
  return pfn_fail(ctx, PFN_ERR_UNSUPPORTED, "path tracer not built yet");
}
extern "C" pfn_status pfn_image_error(pfn_context *ctx, const float *, const float *, int64_t,
                                      double *, double *, double *) {
  if (!ctx) return PFN_ERR_INVALID_ARG;
  return pfn_fail(ctx, PFN_ERR_UNSUPPORTED, "not built yet");
}
