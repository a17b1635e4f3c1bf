// Monte Carlo volumetric path tracer (the full-GI baseline of Section 4.3) and FP64 image
// error reductions.
//
// One lane per pixel, looping over its samples: delta tracking (Woodcock) with the global
// majorant finds real collisions; at each collision, next-event estimation toward every selected
// point light with a ratio-tracking transmittance estimate; the throughput takes the albedo and
// the direction is resampled from HG(g); at most max_bounces collisions, optional Russian
// roulette.  Black background.  Samples are split over launches so that no launch runs long.
#include <mutex>
#include <string>

#include "pfn_ctx.h"

#define PT_THREADS 256

struct PtArgs {
  const void *vol;
  BrickGrid vg;
  const float4 *tf;
  float ext_scale, majorant;
  int n_lights, light_mask;
  float light_pos[4][3], light_int[4][3];
  float eye[3], fwd[3], right[3], up[3];
  int width, height;
  int spp_total, s_begin, s_end;
  int max_bounces, rr_start;
  float g;
  uint64_t seed;
  float *out;
  int first;  // first launch writes, later launches add
  float scale;  // applied on the last launch (1 / spp_total), else 1
};

template <typename VT>
__device__ float ratio_tracking(const PtArgs &a, const float4 *tf, f3 x, f3 p, Philox &rng) {
  f3 v = p - x;
  float dist = sqrtf(dot(v, v));
  f3 d = v * (1.0f / dist);
  float tmax = fminf(dist, exit_distance(x, d));
  float T = 1.0f, t = 0.0f;
  if (!(a.majorant > 0.0f)) return 1.0f;
  const VT *vol = reinterpret_cast<const VT *>(a.vol);
  for (;;) {
    t += -logf(rng.next()) / a.majorant;
    if (t >= tmax) break;
    float sig = tf_lookup(tf, density_at(vol, a.vg, x + d * t)).w * a.ext_scale;
    T *= 1.0f - sig / a.majorant;
  }
  return T;
}

template <typename VT>
__global__ __launch_bounds__(PT_THREADS) void pt_kernel(PtArgs a) {
  __shared__ float4 tf[256];
  for (int i = threadIdx.x; i < 256; i += blockDim.x) tf[i] = a.tf[i];
  __syncthreads();
  const int64_t pix = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pix >= (int64_t)a.width * a.height) return;
  const int px = (int)(pix % a.width), py = (int)(pix / a.width);
  const VT *vol = reinterpret_cast<const VT *>(a.vol);
  const f3 eye = {a.eye[0], a.eye[1], a.eye[2]};
  const f3 fw = {a.fwd[0], a.fwd[1], a.fwd[2]};
  const f3 rt = {a.right[0], a.right[1], a.right[2]};
  const f3 up = {a.up[0], a.up[1], a.up[2]};
  f3 acc = {0.f, 0.f, 0.f};
  for (int s = a.s_begin; s < a.s_end; ++s) {
    Philox rng;
    rng.init(a.seed, (uint64_t)pix * (uint64_t)a.spp_total + (uint64_t)s, STREAM_PT);
    float jx = rng.next(), jy = rng.next();
    float sx = 2.0f * ((float)px + jx) / (float)a.width - 1.0f;
    float sy = 1.0f - 2.0f * ((float)py + jy) / (float)a.height;
    f3 d = normalize3(fw + rt * sx + up * sy);
    f3 o = eye;
    float t, tmax;
    if (!clip_cube(o, d, t, tmax)) continue;
    if (!(a.majorant > 0.0f)) continue;
    f3 beta = {1.f, 1.f, 1.f};
    int k = 0;
    for (;;) {
      t += -logf(rng.next()) / a.majorant;
      if (t >= tmax) break;
      f3 x = o + d * t;
      float4 op = tf_lookup(tf, density_at(vol, a.vg, x));
      float sig = op.w * a.ext_scale;
      if (!(rng.next() < sig / a.majorant)) continue;
      ++k;
      f3 alb = {op.x, op.y, op.z};
      for (int l = 0; l < a.n_lights; ++l) {
        if (!((a.light_mask >> l) & 1)) continue;
        f3 p = {a.light_pos[l][0], a.light_pos[l][1], a.light_pos[l][2]};
        f3 v = x - p;
        float r2 = dot(v, v);
        float mu = -dot(v, d) / sqrtf(r2);
        float T = ratio_tracking<VT>(a, tf, x, p, rng);
        float wgt = hg_eval(a.g, mu) * T / r2;
        f3 I = {a.light_int[l][0], a.light_int[l][1], a.light_int[l][2]};
        acc = acc + mul(mul(beta, alb), I) * wgt;
      }
      beta = mul(beta, alb);
      if (k >= a.max_bounces) break;
      float u1 = rng.next(), u2 = rng.next();
      d = hg_sample_dir(a.g, d, u1, u2);
      if (a.rr_start > 0 && k >= a.rr_start) {
        float q = fminf(1.0f, maxc(beta));
        if (!(rng.next() < q)) break;
        beta = beta * (1.0f / q);
      }
      o = x;
      t = 0.0f;
      tmax = exit_distance(o, d);
    }
  }
  float *op = a.out + pix * 3;
  if (a.first) {
    op[0] = acc.x * a.scale;
    op[1] = acc.y * a.scale;
    op[2] = acc.z * a.scale;
  } else {
    op[0] = (op[0] + acc.x) * a.scale;
    op[1] = (op[1] + acc.y) * a.scale;
    op[2] = (op[2] + acc.z) * a.scale;
  }
}

extern "C" pfn_status pfn_render_path_traced(pfn_context *ctx, const pfn_camera *c, int spp,
                                             int max_bounces, float g, int rr_start,
                                             int light_mask, uint64_t seed, float *out) {
  if (!ctx) return PFN_ERR_INVALID_ARG;
  if (!c || !out) return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "NULL argument");
  if (c->width < 1 || c->height < 1 || c->width > 16384 || c->height > 16384)
    return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "image sizes in [1, 16384]");
  if (!(c->fov_y_deg > 0.0f && c->fov_y_deg < 179.0f))
    return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "fov_y in (0, 179)");
  if (spp < 1 || spp > (1 << 20)) return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "spp in [1, 2^20]");
  if (max_bounces < 1 || max_bounces > 1024)
    return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "max_bounces in [1, 1024]");
  if (!(std::fabs(g) <= 0.95f)) return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "|g| <= 0.95");
  if (light_mask < 0 || light_mask >= 16)
    return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "light_mask in [0, 16)");
  if (!ctx->vol || !ctx->tf_set || ctx->n_lights < 1)
    return pfn_fail(ctx, PFN_ERR_NOT_READY, "path tracing needs volume, transfer function, lights");
  PFN_HIP(ctx, hipSetDevice(ctx->device));
  PtArgs a{};
  a.vol = ctx->vol;
  a.vg = ctx->vol_grid;
  a.tf = ctx->tf_dev;
  a.ext_scale = ctx->ext_scale;
  a.majorant = ctx->majorant;
  a.n_lights = ctx->n_lights;
  a.light_mask = light_mask == 0 ? 0xF : light_mask;
  for (int l = 0; l < ctx->n_lights; ++l)
    for (int k = 0; k < 3; ++k) {
      a.light_pos[l][k] = ctx->lights[l].pos[k];
      a.light_int[l][k] = ctx->lights[l].intensity[k];
    }
  double e[3] = {c->eye[0], c->eye[1], c->eye[2]};
  double f[3] = {c->target[0] - e[0], c->target[1] - e[1], c->target[2] - e[2]};
  double fn = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  if (!(fn > 0.0)) return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "camera target equals eye");
  for (double &v : f) v /= fn;
  double r[3] = {f[1] * c->up[2] - f[2] * c->up[1], f[2] * c->up[0] - f[0] * c->up[2],
                 f[0] * c->up[1] - f[1] * c->up[0]};
  double rn = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  if (!(rn > 1e-9)) return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "up is parallel to the view");
  for (double &v : r) v /= rn;
  double u[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]};
  double th = std::tan(0.5 * (double)c->fov_y_deg * M_PI / 180.0);
  double aspect = (double)c->width / (double)c->height;
  for (int k = 0; k < 3; ++k) {
    a.eye[k] = (float)e[k];
    a.fwd[k] = (float)f[k];
    a.right[k] = (float)(r[k] * th * aspect);
    a.up[k] = (float)(u[k] * th);
  }
  a.width = c->width;
  a.height = c->height;
  a.spp_total = spp;
  a.max_bounces = max_bounces;
  a.rr_start = rr_start;
  a.g = g;
  a.seed = seed;
  a.out = out;
  const int64_t npix = (int64_t)c->width * c->height;
  // keep each launch to about 2^27 pixel-samples
  int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(spp, ((int64_t)1 << 27) / npix));
  unsigned blocks = (unsigned)((npix + PT_THREADS - 1) / PT_THREADS);
  const int tslot = timing_begin(ctx);
  for (int s0 = 0; s0 < spp; s0 += chunk) {
    a.s_begin = s0;
    a.s_end = std::min(spp, s0 + chunk);
    a.first = s0 == 0;
    a.scale = a.s_end == spp ? 1.0f / (float)spp : 1.0f;
    if (ctx->vol_dtype == PFN_F16)
      hipLaunchKernelGGL(pt_kernel<__half>, dim3(blocks), dim3(PT_THREADS), 0, ctx->stream, a);
    else
      hipLaunchKernelGGL(pt_kernel<float>, dim3(blocks), dim3(PT_THREADS), 0, ctx->stream, a);
    PFN_HIP(ctx, hipGetLastError());
  }
  timing_end(ctx, tslot, TK_PT);
  return PFN_OK;
}

// ------------------------------------------------------------------ FP64 error reductions
__global__ void image_error_kernel(const float *__restrict__ img, const float *__restrict__ ref,
                                   int64_t n, double *acc, unsigned *mx) {
  double se = 0.0, sr = 0.0;
  float m = 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double d = (double)img[i] - (double)ref[i];
    se += d * d;
    sr += (double)ref[i];
    m = fmaxf(m, ref[i]);
  }
  for (int off = 32; off > 0; off >>= 1) {
    se += __shfl_down(se, off);
    sr += __shfl_down(sr, off);
    m = fmaxf(m, __shfl_down(m, off));
  }
  if (lane_id() == 0) {
    atomicAdd(&acc[0], se);
    atomicAdd(&acc[1], sr);
    atomicMax(mx, __float_as_uint(fmaxf(m, 0.0f)));
  }
}

extern "C" pfn_status pfn_image_error(pfn_context *ctx, const float *img, const float *ref, int64_t n,
                                      double *rmse, double *rel, double *psnr) {
  if (!ctx) return PFN_ERR_INVALID_ARG;
  if (!img || !ref || n < 1) return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "bad image arguments");
  PFN_HIP(ctx, hipSetDevice(ctx->device));
  pfn_status st = ensure_scratch(ctx, 64);
  if (st) return st;
  double *acc = (double *)ctx->scratch;
  unsigned *mx = (unsigned *)(acc + 2);
  PFN_HIP(ctx, hipMemsetAsync(acc, 0, 32, ctx->stream));
  unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(image_error_kernel, dim3(blocks), dim3(256), 0, ctx->stream, img, ref, n, acc, mx);
  PFN_HIP(ctx, hipGetLastError());
  double h[3];
  PFN_HIP(ctx, hipMemcpyAsync(h, acc, 24, hipMemcpyDeviceToHost, ctx->stream));
  PFN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  unsigned mbits;
  std::memcpy(&mbits, &h[2], 4);
  float m;
  std::memcpy(&m, &mbits, 4);
  double r = std::sqrt(h[0] / (double)n);
  if (rmse) *rmse = r;
  if (rel) *rel = r / (h[1] / (double)n);
  if (psnr) *psnr = 20.0 * std::log10((double)m / r);
  return PFN_OK;
}

// ------------------------------------------------------------------ error reduction without allocation
// pfn_image_error_noalloc keeps its partial sums in this fixed device array instead of a
// context buffer.  Host code never uses the array's name as an address: each device's copy is
// resolved once with hipGetSymbolAddress (pfn_noalloc_init, called by pfn_create with the device
// current) and that pointer is what the kernels receive.
#define NOALLOC_MAX_BLOCKS 2048
#define NOALLOC_ITEMS 64  // values per thread of the partial-sum kernel
static __device__ __align__(256) double scratch[NOALLOC_MAX_BLOCKS * 4];

#define NOALLOC_MAX_DEVICES 64
static std::mutex g_noalloc_mu;
static void *g_noalloc_ptr[NOALLOC_MAX_DEVICES];

hipError_t pfn_noalloc_init(int device) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (g_noalloc_ptr[device]) return hipSuccess;
  void *p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_noalloc_ptr[device] = p;
  return hipSuccess;
}

// Per block: sum of squared differences, sum of the reference and its maximum over the block's
// 256 * NOALLOC_ITEMS values (written, not accumulated: nothing needs clearing).
__global__ __launch_bounds__(256) void image_error_partial_kernel(const float *__restrict__ img,
                                                                  const float *__restrict__ ref,
                                                                  int64_t n, double *part) {
  __shared__ double sse[4], ssr[4];
  __shared__ float smx[4];
  double se = 0.0, sr = 0.0;
  float m = 0.0f;
  const int64_t base = (int64_t)blockIdx.x * (256 * NOALLOC_ITEMS) + threadIdx.x;
  for (int k = 0; k < NOALLOC_ITEMS; ++k) {
    const int64_t i = base + (int64_t)k * 256;
    if (i < n) {
      const double d = (double)img[i] - (double)ref[i];
      se += d * d;
      sr += (double)ref[i];
      m = fmaxf(m, ref[i]);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    se += __shfl_down(se, off);
    sr += __shfl_down(sr, off);
    m = fmaxf(m, __shfl_down(m, off));
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sse[w] = se;
    ssr[w] = sr;
    smx[w] = m;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double* o = part + 4 * (size_t)blockIdx.x;
    o[0] = (sse[0] + sse[1]) + (sse[2] + sse[3]);
    o[1] = (ssr[0] + ssr[1]) + (ssr[2] + ssr[3]);
    o[2] = (double)fmaxf(fmaxf(smx[0], smx[1]), fmaxf(smx[2], smx[3]));
    o[3] = 0.0;
  }
}

// One block adds the partials in a fixed order and writes (RMSE, RMSE / mean(ref), PSNR).
__global__ __launch_bounds__(256) void image_error_final_kernel(const double *part, int nblocks,
                                                                int64_t n, double *result) {
  __shared__ double sse[256], ssr[256], smx[256];
  double se = 0.0, sr = 0.0, m = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += 256) {
    se += part[4 * b];
    sr += part[4 * b + 1];
    m = fmax(m, part[4 * b + 2]);
  }
  sse[threadIdx.x] = se;
  ssr[threadIdx.x] = sr;
  smx[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sse[threadIdx.x] += sse[threadIdx.x + s];
      ssr[threadIdx.x] += ssr[threadIdx.x + s];
      smx[threadIdx.x] = fmax(smx[threadIdx.x], smx[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double r = sqrt(sse[0] / (double)n);
    result[0] = r;
    result[1] = r / (ssr[0] / (double)n);
    result[2] = 20.0 * log10(smx[0] / r);
  }
}

extern "C" pfn_status pfn_image_error_noalloc(pfn_context *ctx, const float *img, const float *ref,
                                              int64_t n, double *dev_result) {
  if (!ctx) return PFN_ERR_INVALID_ARG;
  if (!img || !ref || !dev_result || n < 1)
    return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "bad image arguments");
  const int64_t max_n = (int64_t)NOALLOC_MAX_BLOCKS * 256 * NOALLOC_ITEMS;
  if (n > max_n)
    return pfn_fail(ctx, PFN_ERR_INVALID_ARG,
                    "n exceeds the no-allocation limit of " + std::to_string(max_n) + " values");
  void *p = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (ctx->device >= 0 && ctx->device < NOALLOC_MAX_DEVICES) p = g_noalloc_ptr[ctx->device];
  }
  if (!p) return pfn_fail(ctx, PFN_ERR_NOT_READY, "no-allocation scratch not resolved");
  PFN_HIP(ctx, hipSetDevice(ctx->device));
  double *part = (double *)p;
  const int nblocks = (int)((n + 256 * NOALLOC_ITEMS - 1) / (256 * NOALLOC_ITEMS));
  hipLaunchKernelGGL(image_error_partial_kernel, dim3((unsigned)nblocks), dim3(256), 0,
                     ctx->stream, img, ref, n, part);
  PFN_HIP(ctx, hipGetLastError());
  hipLaunchKernelGGL(image_error_final_kernel, dim3(1), dim3(256), 0, ctx->stream, part, nblocks,
                     n, dev_result);
  PFN_HIP(ctx, hipGetLastError());
  return PFN_OK;
}
