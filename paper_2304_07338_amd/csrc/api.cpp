// C ABI of the library: argument validation, context-owned buffers and kernel dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "march.h"
#include "pfn_ctx.h"

// ------------------------------------------------------------------ errors and helpers
pfn_status pfn_fail(pfn_context *ctx, pfn_status st, const std::string &msg) {
  if (ctx) ctx->err = msg;
  return st;
}

pfn_status pfn_hip(pfn_context *ctx, hipError_t e, const char *what) {
  // The runtime also keeps a failed call's status as its "last error"; clear it, so that the
  // launch checks of later calls (hipGetLastError after a kernel launch) do not report it
  // again.  A sticky device error is reported again by the runtime's next call anyway.
  (void)hipGetLastError();
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    return pfn_fail(ctx, PFN_ERR_OUT_OF_MEMORY, m);
  return pfn_fail(ctx, PFN_ERR_HIP, m);
}

#define CHECK_CTX(ctx) \
  if (!(ctx)) return PFN_ERR_INVALID_ARG
#define ARG(cond, msg) \
  if (!(cond)) return pfn_fail(ctx, PFN_ERR_INVALID_ARG, msg)

static hipError_t dev_alloc(void **p, size_t bytes) {
  if (bytes == 0) bytes = 16;
  return hipMalloc(p, bytes);
}
template <typename T>
static void dev_free(T *&p) {
  if (p) (void)hipFree((void *)p);
  p = nullptr;
}

pfn_status ensure_scratch(pfn_context *ctx, size_t bytes) {
  if (ctx->scratch_bytes >= bytes) return PFN_OK;
  dev_free(ctx->scratch);
  ctx->scratch_bytes = 0;
  PFN_HIP(ctx, dev_alloc(&ctx->scratch, bytes));
  ctx->scratch_bytes = bytes;
  return PFN_OK;
}

// Pending event pairs are collected once none is open (when the totals are read, or when the
// pool is full at the next opening).
static void timing_collect(pfn_context *ctx) {
  if (ctx->ev_open > 0) return;
  for (int i = 0; i < ctx->ev_pending; ++i) {
    hipEvent_t a = ctx->ev_pool[2 * i], b = ctx->ev_pool[2 * i + 1];
    if (ctx->ev_kernel[i] < 0 || hipEventSynchronize(b) != hipSuccess) continue;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, a, b) == hipSuccess) {
      ctx->t_ms[ctx->ev_kernel[i]] += ms;
      ctx->t_n[ctx->ev_kernel[i]] += 1;
    }
  }
  ctx->ev_pending = 0;
}

// Opens an event pair on the context's stream before a launch; the host does not wait here.
// Returns the pair's slot (-1 when timing is off); pairs may nest.
int timing_begin(pfn_context *ctx) { return timing_begin_on(ctx, ctx->stream); }
void timing_end(pfn_context *ctx, int slot, int kernel) {
  timing_end_on(ctx, slot, kernel, ctx->stream);
}

int timing_begin_on(pfn_context *ctx, hipStream_t stream) {
  if (!ctx->timing) return -1;
  if (ctx->ev_pending >= 512) timing_collect(ctx);
  int i = ctx->ev_pending;
  while ((int)ctx->ev_pool.size() < 2 * (i + 1)) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    ctx->ev_pool.push_back(e);
    if (ctx->ev_kernel.size() * 2 < ctx->ev_pool.size()) ctx->ev_kernel.push_back(-1);
  }
  if (hipEventRecord(ctx->ev_pool[2 * i], stream) != hipSuccess) return -1;
  ctx->ev_kernel[i] = -1;
  ctx->ev_pending = i + 1;
  ctx->ev_open += 1;
  return i;
}

void timing_end_on(pfn_context *ctx, int slot, int kernel, hipStream_t stream) {
  if (slot < 0 || !ctx->timing) return;
  (void)hipEventRecord(ctx->ev_pool[2 * slot + 1], stream);
  ctx->ev_kernel[slot] = kernel;
  ctx->ev_open -= 1;
}

static bool finite3(const float *v) {
  return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]);
}

// ------------------------------------------------------------------ context
extern "C" pfn_status pfn_create(int device, void *hip_stream, pfn_context **out) {
  if (!out) return PFN_ERR_INVALID_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n == 0) return PFN_ERR_HIP;
  if (device < 0 || device >= n) return PFN_ERR_INVALID_ARG;
  if (hipSetDevice(device) != hipSuccess) return PFN_ERR_HIP;
  // once per device: the device address of pfn_image_error_noalloc's fixed scratch array
  if (pfn_noalloc_init(device) != hipSuccess) {
    (void)hipGetLastError();
    return PFN_ERR_HIP;
  }
  pfn_context *ctx = new (std::nothrow) pfn_context();
  if (!ctx) return PFN_ERR_OUT_OF_MEMORY;
  ctx->device = device;
  // NULL selects the device's null stream, which orders the library's work with every other
  // user of that stream (e.g. PyTorch's default stream)
  ctx->stream = (hipStream_t)hip_stream;
  *out = ctx;
  return PFN_OK;
}

static void free_field(FieldSlot &f) {
  dev_free(f.master);
  dev_free(f.adam_m);
  dev_free(f.adam_v);
  dev_free(f.grad);
  for (int p = 0; p < 3; ++p) {
    dev_free(f.lp_table[p]);
    dev_free(f.mlp_packed[p]);
    dev_free(f.mlp_bwd[p]);
    f.lp_valid[p] = false;
    f.bwd_valid[p] = false;
  }
  f.init = false;
}

extern "C" void pfn_destroy(pfn_context *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  dev_free(ctx->vol);
  dev_free(ctx->qvol);
  dev_free(ctx->cvol);
  dev_free(ctx->tf_dev);
  dev_free(ctx->lightvol);
  dev_free(ctx->lquad);
  dev_free(ctx->cache);
  dev_free(ctx->rec_x);
  dev_free(ctx->rec_w);
  dev_free(ctx->rec_p);
  dev_free(ctx->rec_bin);
  dev_free(ctx->rec_cnt);
  for (auto &f : ctx->fields) free_field(f);
  dev_free(ctx->scratch);
  dev_free(ctx->train_act);
  dev_free(ctx->jobs_dev);
  dev_free(ctx->fields_dev);
  dev_free(ctx->mlp_ptrs_dev);
  dev_free(ctx->counters);
  dev_free(ctx->queues);
  wf_release(ctx->wf);
  pm_release(ctx->pmap);
  dev_free(ctx->pm_batch);
  for (auto &g : ctx->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  ctx->graphs.clear();
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  delete ctx;
}

extern "C" const char *pfn_last_error(const pfn_context *ctx) {
  if (!ctx) return "null context";
  return ctx->err.c_str();
}

extern "C" pfn_status pfn_sync(pfn_context *ctx) {
  CHECK_CTX(ctx);
  PFN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return PFN_OK;
}

extern "C" pfn_status pfn_set_stream(pfn_context *ctx, void *hip_stream) {
  CHECK_CTX(ctx);
  PFN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  ctx->stream = (hipStream_t)hip_stream;
  return PFN_OK;
}

// ------------------------------------------------------------------ scene
static BrickGrid make_brick_grid(int nx, int ny, int nz, size_t *elems) {
  int bx = (nx + 7) / 8, by = (ny + 7) / 8, bz = (nz + 7) / 8;
  BrickGrid g{nx, ny, nz, bx * 512, bx * by * 512};
  *elems = (size_t)bx * by * bz * 512;
  return g;
}

extern "C" pfn_status pfn_set_volume(pfn_context *ctx, const void *dev_density, pfn_dtype dtype,
                                     int nx, int ny, int nz) {
  CHECK_CTX(ctx);
  ARG(dev_density, "density pointer is NULL");
  ARG(dtype == PFN_F32 || dtype == PFN_F16, "volume dtype must be F32 or F16");
  ARG(nx >= 2 && ny >= 2 && nz >= 2 && nx <= 4096 && ny <= 4096 && nz <= 4096,
      "volume sizes must be in [2, 4096]");
  size_t elems = 0, qe = 0;
  BrickGrid g = make_brick_grid(nx, ny, nz, &elems);
  const BrickGrid qg = make_brick_grid(nx + 1, ny + 1, nz, &qe);
  ARG(elems < ((size_t)1 << 31) && (dtype != PFN_F16 || qe < ((size_t)1 << 31)),
      "volume too large for 32-bit brick offsets");
  PFN_HIP(ctx, hipSetDevice(ctx->device));
  size_t es = dtype == PFN_F16 ? 2 : 4;
  if (!ctx->vol || ctx->vol_elems * (ctx->vol_dtype == PFN_F16 ? 2 : 4) < elems * es) {
    dev_free(ctx->vol);
    PFN_HIP(ctx, dev_alloc(&ctx->vol, elems * es));
  }
  PFN_HIP(ctx, hipMemsetAsync(ctx->vol, 0, elems * es, ctx->stream));
  ctx->vol_grid = g;
  ctx->vol_elems = elems;
  ctx->vol_dtype = dtype;
  ctx->nmax = std::max(nx, std::max(ny, nz));
  PFN_HIP(ctx, launch_brick_volume(ctx, dev_density, dtype, nx, ny, nz));
  if (dtype == PFN_F16) {
    // the march kernels' two-load density lookups (8 bytes per cell, 4x the volume)
    if (!ctx->qvol || ctx->qvol_elems < qe) {
      dev_free(ctx->qvol);
      ctx->qvol = nullptr;
      ctx->qvol_elems = 0;
      PFN_HIP(ctx, dev_alloc((void **)&ctx->qvol, qe * sizeof(uint2)));
      ctx->qvol_elems = qe;
    }
    ctx->qvol_grid = qg;
    PFN_HIP(ctx, launch_quad_volume(ctx));
  } else {
    dev_free(ctx->qvol);
    ctx->qvol = nullptr;
    ctx->qvol_elems = 0;
  }
  ctx->cvol_valid = false;
  if (dtype != PFN_F16) {
    dev_free(ctx->cvol);
    ctx->cvol = nullptr;
    ctx->cvol_elems = 0;
  }
  ctx->lv_valid = false;
  return PFN_OK;
}

extern "C" pfn_status pfn_set_transfer_function(pfn_context *ctx, const float *rgba,
                                                float extinction_scale) {
  CHECK_CTX(ctx);
  ARG(rgba, "transfer function is NULL");
  ARG(std::isfinite(extinction_scale) && extinction_scale >= 0.0f,
      "extinction scale must be finite and >= 0");
  float amax = 0.0f;
  for (int i = 0; i < 1024; ++i) {
    ARG(std::isfinite(rgba[i]) && rgba[i] >= 0.0f && rgba[i] <= 1.0f,
        "transfer function values must be in [0,1]");
    if (i % 4 == 3) amax = std::max(amax, rgba[i]);
  }
  PFN_HIP(ctx, hipSetDevice(ctx->device));
  if (!ctx->tf_dev) PFN_HIP(ctx, dev_alloc((void **)&ctx->tf_dev, 256 * sizeof(float4)));
  std::memcpy(ctx->tf_host, rgba, sizeof(ctx->tf_host));
  PFN_HIP(ctx, hipMemcpyAsync(ctx->tf_dev, ctx->tf_host, sizeof(ctx->tf_host),
                              hipMemcpyHostToDevice, ctx->stream));
  PFN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  ctx->ext_scale = extinction_scale;
  ctx->majorant = amax * extinction_scale;
  ctx->tf_set = true;
  ctx->lv_valid = false;
  return PFN_OK;
}

extern "C" pfn_status pfn_set_lights(pfn_context *ctx, const pfn_point_light *lights, int n) {
  CHECK_CTX(ctx);
  ARG(lights, "lights pointer is NULL");
  ARG(n >= 1 && n <= PFN_MAX_LIGHTS, "1 to 4 lights");
  for (int l = 0; l < n; ++l) {
    ARG(finite3(lights[l].pos) && finite3(lights[l].intensity), "light values must be finite");
    ARG(lights[l].intensity[0] >= 0 && lights[l].intensity[1] >= 0 && lights[l].intensity[2] >= 0,
        "light intensity must be >= 0");
  }
  for (int l = 0; l < n; ++l) ctx->lights[l] = lights[l];
  ctx->n_lights = n;
  ctx->lv_valid = false;
  return PFN_OK;
}

static pfn_status need_scene(pfn_context *ctx) {
  if (!ctx->vol) return pfn_fail(ctx, PFN_ERR_NOT_READY, "no volume set");
  if (!ctx->tf_set) return pfn_fail(ctx, PFN_ERR_NOT_READY, "no transfer function set");
  if (ctx->n_lights < 1) return pfn_fail(ctx, PFN_ERR_NOT_READY, "no lights set");
  return PFN_OK;
}

extern "C" pfn_status pfn_build_light_volume(pfn_context *ctx, float step_voxels) {
  CHECK_CTX(ctx);
  ARG(std::isfinite(step_voxels) && step_voxels > 0.0f && step_voxels <= 64.0f,
      "step_voxels must be in (0, 64]");
  pfn_status st = need_scene(ctx);
  if (st) return st;
  PFN_HIP(ctx, hipSetDevice(ctx->device));
  const BrickGrid &v = ctx->vol_grid;
  size_t elems = 0;
  BrickGrid g = make_brick_grid((v.nx + 1) / 2, (v.ny + 1) / 2, (v.nz + 1) / 2, &elems);
  if (!ctx->lightvol || ctx->lv_elems < elems) {
    dev_free(ctx->lightvol);
    PFN_HIP(ctx, dev_alloc((void **)&ctx->lightvol, elems * sizeof(ushort4)));
  }
  ctx->lv_grid = g;
  ctx->lv_elems = elems;
  PFN_HIP(ctx, hipMemsetAsync(ctx->lightvol, 0, elems * sizeof(ushort4), ctx->stream));
  if (ctx->vol_dtype == PFN_F16 && !ctx->cvol_valid) {
    // the light march's one-load density lookups (16 bytes per cell, 8x the volume), kept while
    // the volume stays; a volume whose copy would pass 32-bit brick offsets, or does not fit in
    // the free device memory, is marched with plain eight-load lookups
    size_t ce = 0;
    const BrickGrid cg = make_brick_grid(v.nx + 1, v.ny + 1, v.nz + 1, &ce);
    if (ce < ((size_t)1 << 31)) {
      if (!ctx->cvol || ctx->cvol_elems < ce) {
        dev_free(ctx->cvol);
        ctx->cvol_elems = 0;
        if (dev_alloc((void **)&ctx->cvol, ce * sizeof(uint4)) == hipSuccess) {
          ctx->cvol_elems = ce;
        } else {
          (void)hipGetLastError();  // an optional copy: clear the failed allocation's error
          ctx->cvol = nullptr;
        }
      }
      if (ctx->cvol) {
        ctx->cvol_grid = cg;
        PFN_HIP(ctx, launch_cube_volume(ctx));
        ctx->cvol_valid = true;
      }
    }
  }
  PFN_HIP(ctx, launch_light_volume(ctx, step_voxels / (float)ctx->nmax));
  ctx->lquad_lights = 0;
  // The march kernels' four-load light lookups (24 bytes per cell) pay while the copy stays
  // near the caches: measured on a 1080p view, equal or 2 % faster with a 256^3 light grid
  // (0.4 GB copy) and 3 % / 18 % slower (field / cache frame, 4 spp) with a 512^3 one (3.2 GB),
  // where the plain 8-byte texels are used instead.
  if (ctx->n_lights <= 3 && (size_t)g.nx * g.ny * g.nz <= ((size_t)1 << 24)) {
    size_t qe = 0;
    const BrickGrid qg = make_brick_grid(g.nx + 1, g.ny + 1, g.nz, &qe);
    if (!ctx->lquad || ctx->lquad_elems < qe) {
      dev_free(ctx->lquad);
      ctx->lquad = nullptr;
      ctx->lquad_elems = 0;
      PFN_HIP(ctx, dev_alloc((void **)&ctx->lquad, qe * 6 * sizeof(uint32_t)));
      ctx->lquad_elems = qe;
    }
    ctx->lquad_grid = qg;
    PFN_HIP(ctx, launch_light_quad(ctx));
    ctx->lquad_lights = ctx->n_lights;
  }
  ctx->lv_valid = true;
  return PFN_OK;
}

extern "C" pfn_status pfn_get_light_volume(pfn_context *ctx, uint16_t *dev_out, size_t n_texels) {
  CHECK_CTX(ctx);
  if (!ctx->lv_valid) return pfn_fail(ctx, PFN_ERR_NOT_READY, "light volume not built");
  const BrickGrid &g = ctx->lv_grid;
  ARG(dev_out, "output is NULL");
  ARG(n_texels == (size_t)g.nx * g.ny * g.nz, "n_texels must equal the grid's texel count");
  PFN_HIP(ctx, hipSetDevice(ctx->device));
  PFN_HIP(ctx, launch_light_unbrick(ctx, dev_out));
  return PFN_OK;
}

// ------------------------------------------------------------------ cache
extern "C" pfn_status pfn_get_cache(pfn_context *ctx, float *dev_out, size_t n_floats) {
  CHECK_CTX(ctx);
  ARG(dev_out, "output is NULL");
  if (!ctx->cache_valid) return pfn_fail(ctx, PFN_ERR_NOT_READY, "no cache");
  size_t cells = (size_t)ctx->cache_res * ctx->cache_res * ctx->cache_res * ctx->cache_bins;
  ARG(n_floats == cells * 3, "n_floats must be n_bins * res^3 * 3");
  PFN_HIP(ctx, launch_cache_unpack(ctx, dev_out, cells));
  return PFN_OK;
}

extern "C" pfn_status pfn_set_cache(pfn_context *ctx, const float *dev_in, int n_bins,
                                    const float *g_bins, int res, double kappa) {
  CHECK_CTX(ctx);
  ARG(dev_in && g_bins, "NULL argument");
  ARG(n_bins >= 1 && n_bins <= 8, "1 to 8 bins");
  ARG(res >= 2 && res <= 512, "cache resolution in [2, 512]");
  ARG(std::isfinite(kappa) && kappa > 0.0, "kappa must be finite and > 0");
  for (int b = 0; b < n_bins; ++b) {
    ARG(std::isfinite(g_bins[b]) && std::fabs(g_bins[b]) <= 0.95f, "|g| <= 0.95");
    if (b) ARG(g_bins[b] > g_bins[b - 1], "g bins must be ascending");
  }
  PFN_HIP(ctx, hipSetDevice(ctx->device));
  pfn_status st = alloc_cache(ctx, n_bins, res);
  if (st) return st;
  for (int b = 0; b < n_bins; ++b) ctx->g_bins[b] = g_bins[b];
  size_t cells = (size_t)res * res * res * n_bins;
  PFN_HIP(ctx, launch_cache_pack(ctx, dev_in, cells));
  ctx->kappa = kappa;
  ctx->cache_valid = true;
  return PFN_OK;
}

pfn_status alloc_cache(pfn_context *ctx, int n_bins, int res) {
  size_t cells = (size_t)res * res * res * n_bins;
  size_t have = (size_t)ctx->cache_res * ctx->cache_res * ctx->cache_res * ctx->cache_bins;
  if (!ctx->cache || have < cells) {
    dev_free(ctx->cache);
    ctx->cache_bins = ctx->cache_res = 0;
    PFN_HIP(ctx, dev_alloc((void **)&ctx->cache, cells * sizeof(float4)));
  }
  ctx->cache_bins = n_bins;
  ctx->cache_res = res;
  return PFN_OK;
}

extern "C" pfn_status pfn_cache_info(pfn_context *ctx, int *n_bins, int *res, double *kappa) {
  CHECK_CTX(ctx);
  if (!ctx->cache_valid) return pfn_fail(ctx, PFN_ERR_NOT_READY, "no cache");
  if (n_bins) *n_bins = ctx->cache_bins;
  if (res) *res = ctx->cache_res;
  if (kappa) *kappa = ctx->kappa;
  return PFN_OK;
}

// ------------------------------------------------------------------ field
extern "C" pfn_status pfn_field_select(pfn_context *ctx, int slot) {
  CHECK_CTX(ctx);
  ARG(slot >= 0 && slot < PFN_MAX_FIELDS, "field slot in [0, 8)");
  ctx->cur_field = slot;
  return PFN_OK;
}

static pfn_status field_layout(pfn_context *ctx, const pfn_field_desc *d, FieldSlot &f) {
  ARG(d->levels >= 1 && d->levels <= PFN_MAX_LEVELS, "levels in [1, 16]");
  ARG(d->feats_per_level == 2 || d->feats_per_level == 8, "feats_per_level must be 2 or 8");
  ARG(d->base_res >= 2 && d->base_res <= 4096, "base_res in [2, 4096]");
  ARG(std::isfinite(d->growth) && d->growth >= 1.0f && d->growth <= 4.0f, "growth in [1, 4]");
  ARG(d->log2_table >= 4 && d->log2_table <= 24, "log2_table in [4, 24]");
  ARG(d->hidden_layers >= 1 && d->hidden_layers <= PFN_MAX_HIDDEN, "hidden_layers in [1, 7]");
  ARG(d->width == PFN_WIDTH, "width must be 64");
  ARG(std::isfinite(d->psi) && d->psi > 0.0f && d->psi <= 12.0f, "psi in (0, 12]");
  f.desc = *d;
  const size_t table = (size_t)1 << d->log2_table;
  double r = (double)d->base_res;
  size_t off = 0, offd = 0;
  f.pos = GridLevels{};
  f.dir = GridLevels{};
  for (int l = 0; l < d->levels; ++l) {
    // FP32 positions carry 24 bits: a finer level could not resolve its cells
    ARG(r < 16777216.0, "level resolution above 2^24");
    int res = (int)std::floor(r);
    size_t d3 = (size_t)(res + 1) * (res + 1) * (res + 1), d2 = (size_t)(res + 1) * (res + 1);
    f.pos.res[l] = res;
    f.pos.off[l] = (uint32_t)off;
    if (d3 <= table) f.pos.dense_mask |= 1u << l;
    off += d3 <= table ? d3 : table;
    f.dir.res[l] = res;
    f.dir.off[l] = (uint32_t)offd;
    if (d2 <= table) f.dir.dense_mask |= 1u << l;
    offd += d2 <= table ? d2 : table;
    r *= (double)d->growth;
  }
  f.pos_entries = off;
  f.dir_entries = offd;
  const int F = d->feats_per_level;
  f.mlp_off = (size_t)F * (off + offd);
  size_t w = f.mlp_off;
  int n_in = 2 * F * d->levels + 1;
  for (int m = 0; m <= d->hidden_layers; ++m) {
    f.w_off[m] = w;
    int rows = (m == d->hidden_layers) ? 3 : d->width;
    int cols = (m == 0) ? n_in : d->width;
    w += (size_t)rows * cols;
  }
  f.n_params = w;
  return PFN_OK;
}

extern "C" pfn_status pfn_field_init(pfn_context *ctx, const pfn_field_desc *desc, uint64_t seed) {
  CHECK_CTX(ctx);
  ARG(desc, "desc is NULL");
  FieldSlot nf;
  pfn_status st = field_layout(ctx, desc, nf);
  if (st) return st;
  PFN_HIP(ctx, hipSetDevice(ctx->device));
  FieldSlot &f = ctx->fields[ctx->cur_field];
  free_field(f);
  f = nf;
  size_t n = f.n_params;
  PFN_HIP(ctx, dev_alloc((void **)&f.master, n * 4));
  PFN_HIP(ctx, dev_alloc((void **)&f.adam_m, n * 4));
  PFN_HIP(ctx, dev_alloc((void **)&f.adam_v, n * 4));
  PFN_HIP(ctx, dev_alloc((void **)&f.grad, n * 4));
  // 16-bit copies: one 32-bit word per pair of features
  size_t entries = (f.pos_entries + f.dir_entries) * (size_t)(desc->feats_per_level / 2);
  for (int p = 1; p <= 2; ++p) PFN_HIP(ctx, dev_alloc((void **)&f.lp_table[p], entries * 4));
  for (int p = 0; p <= 2; ++p)
    PFN_HIP(ctx, dev_alloc(&f.mlp_packed[p],
                           (size_t)mlp_packed_elems(p, desc->hidden_layers,
                                                    desc->feats_per_level / 2) * (p ? 2 : 4)));
  PFN_HIP(ctx, hipMemsetAsync(f.adam_m, 0, n * 4, ctx->stream));
  PFN_HIP(ctx, hipMemsetAsync(f.adam_v, 0, n * 4, ctx->stream));
  PFN_HIP(ctx, hipMemsetAsync(f.grad, 0, n * 4, ctx->stream));
  PFN_HIP(ctx, launch_field_init(ctx, f, seed));
  f.adam_t = 0;
  f.kappa = ctx->cache_valid ? ctx->kappa : 1.0;
  f.init = true;
  return PFN_OK;
}

static pfn_status need_field(pfn_context *ctx, int slot) {
  if (!ctx->fields[slot].init)
    return pfn_fail(ctx, PFN_ERR_NOT_READY, "field slot " + std::to_string(slot) + " not initialised");
  return PFN_OK;
}

pfn_status field_refresh(pfn_context *ctx, FieldSlot &f, int prec) {
  if (f.lp_valid[prec]) return PFN_OK;
  PFN_HIP(ctx, launch_field_pack(ctx, f, prec));
  f.lp_valid[prec] = true;
  return PFN_OK;
}

void field_params_changed(FieldSlot &f) {
  for (int p = 0; p < 3; ++p) {
    f.lp_valid[p] = false;
    f.bwd_valid[p] = false;
  }
}

extern "C" pfn_status pfn_field_num_params(pfn_context *ctx, size_t *n) {
  CHECK_CTX(ctx);
  ARG(n, "output is NULL");
  pfn_status st = need_field(ctx, ctx->cur_field);
  if (st) return st;
  *n = ctx->fields[ctx->cur_field].n_params;
  return PFN_OK;
}

extern "C" pfn_status pfn_field_get_params(pfn_context *ctx, float *dev_out, size_t n) {
  CHECK_CTX(ctx);
  ARG(dev_out, "output is NULL");
  pfn_status st = need_field(ctx, ctx->cur_field);
  if (st) return st;
  FieldSlot &f = ctx->fields[ctx->cur_field];
  ARG(n == f.n_params, "n must equal the parameter count");
  PFN_HIP(ctx, hipMemcpyAsync(dev_out, f.master, n * 4, hipMemcpyDeviceToDevice, ctx->stream));
  return PFN_OK;
}

extern "C" pfn_status pfn_field_set_params(pfn_context *ctx, const float *dev_in, size_t n) {
  CHECK_CTX(ctx);
  ARG(dev_in, "input is NULL");
  pfn_status st = need_field(ctx, ctx->cur_field);
  if (st) return st;
  FieldSlot &f = ctx->fields[ctx->cur_field];
  ARG(n == f.n_params, "n must equal the parameter count");
  PFN_HIP(ctx, hipMemcpyAsync(f.master, dev_in, n * 4, hipMemcpyDeviceToDevice, ctx->stream));
  field_params_changed(f);
  return PFN_OK;
}

extern "C" pfn_status pfn_field_set_kappa(pfn_context *ctx, double kappa) {
  CHECK_CTX(ctx);
  ARG(std::isfinite(kappa) && kappa > 0.0, "kappa must be finite and > 0");
  pfn_status st = need_field(ctx, ctx->cur_field);
  if (st) return st;
  ctx->fields[ctx->cur_field].kappa = kappa;
  return PFN_OK;
}

static int prec_of(pfn_dtype d) { return d == PFN_F32 ? P_F32 : d == PFN_BF16 ? P_BF16 : P_F16; }

extern "C" pfn_status pfn_field_query(pfn_context *ctx, pfn_dtype precision, const float *xyz,
                                      const float *dir, const float *g, int64_t n, float *lp,
                                      float *rgb) {
  CHECK_CTX(ctx);
  ARG(precision == PFN_F32 || precision == PFN_F16 || precision == PFN_BF16, "bad precision");
  ARG(n >= 0 && n < ((int64_t)1 << 38), "n out of range");
  ARG(n == 0 || (xyz && dir && g && lp), "NULL argument");
  pfn_status st = need_field(ctx, ctx->cur_field);
  if (st) return st;
  if (n == 0) return PFN_OK;
  PFN_HIP(ctx, hipSetDevice(ctx->device));
  FieldSlot &f = ctx->fields[ctx->cur_field];
  int p = prec_of(precision);
  st = field_refresh(ctx, f, p);
  if (st) return st;
  const int tslot = timing_begin(ctx);
  PFN_HIP(ctx, launch_field_query(ctx, f, p, xyz, dir, g, n, lp, rgb));
  timing_end(ctx, tslot, TK_QUERY);
  return PFN_OK;
}

// ------------------------------------------------------------------ rendering
static pfn_status check_camera(pfn_context *ctx, const pfn_camera *c) {
  ARG(c, "camera is NULL");
  ARG(finite3(c->eye) && finite3(c->target) && finite3(c->up), "camera vectors must be finite");
  ARG(std::isfinite(c->fov_y_deg) && c->fov_y_deg > 0.0f && c->fov_y_deg < 179.0f,
      "fov_y in (0, 179)");
  ARG(c->width >= 1 && c->height >= 1 && c->width <= 16384 && c->height <= 16384,
      "image sizes in [1, 16384]");
  double f[3] = {(double)c->target[0] - c->eye[0], (double)c->target[1] - c->eye[1],
                 (double)c->target[2] - c->eye[2]};
  double fn = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  ARG(fn > 0.0, "camera target equals eye");
  double r[3] = {f[1] * c->up[2] - f[2] * c->up[1], f[2] * c->up[0] - f[0] * c->up[2],
                 f[0] * c->up[1] - f[1] * c->up[0]};
  ARG(std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]) > 1e-9 * fn, "up is parallel to the view");
  return PFN_OK;
}

static pfn_status check_render_params(pfn_context *ctx, const pfn_render_params *p) {
  ARG(p, "render params are NULL");
  ARG(p->spp >= 1 && p->spp <= 65536, "spp in [1, 65536]");
  ARG(std::isfinite(p->step_voxels) && p->step_voxels > 0.0f && p->step_voxels <= 64.0f,
      "step_voxels in (0, 64]");
  ARG(p->max_steps >= 0, "max_steps >= 0");
  ARG(std::isfinite(p->t_min) && p->t_min >= 0.0f && p->t_min < 1.0f, "t_min in [0, 1)");
  ARG(p->field_stride >= 1 && p->field_stride <= 1024, "field_stride in [1, 1024]");
  ARG(std::isfinite(p->g) && std::fabs(p->g) <= 0.95f, "|g| <= 0.95");
  ARG(p->indirect == PFN_INDIRECT_NONE || p->indirect == PFN_INDIRECT_CACHE ||
          p->indirect == PFN_INDIRECT_FIELD,
      "bad indirect mode");
  ARG(p->direct == PFN_DIRECT_SHADOW_RAYS || p->direct == PFN_DIRECT_LIGHT_VOLUME, "bad direct mode");
  ARG(p->field_precision == PFN_F32 || p->field_precision == PFN_F16 ||
          p->field_precision == PFN_BF16,
      "bad field precision");
  ARG(p->light_mask >= 0 && p->light_mask < 16, "light_mask in [0, 16)");
  ARG(p->field_slot >= 0 && p->field_slot < PFN_MAX_FIELDS, "field_slot in [0, 8)");
  if (p->direct == PFN_DIRECT_LIGHT_VOLUME && !ctx->lv_valid)
    return pfn_fail(ctx, PFN_ERR_NOT_READY, "light volume not built (or invalidated)");
  if (p->indirect == PFN_INDIRECT_CACHE && !ctx->cache_valid)
    return pfn_fail(ctx, PFN_ERR_NOT_READY, "no photon cache");
  if (p->indirect == PFN_INDIRECT_FIELD) {
    pfn_status st = need_field(ctx, p->field_slot);
    if (st) return st;
  }
  return PFN_OK;
}

static void fill_job(pfn_context *ctx, const pfn_camera *c, const pfn_render_params *p, float *out,
                     const TileConfig &tc, MarchJob &j) {
  double e[3] = {c->eye[0], c->eye[1], c->eye[2]};
  double f[3] = {c->target[0] - e[0], c->target[1] - e[1], c->target[2] - e[2]};
  double fn = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  for (double &v : f) v /= fn;
  double r[3] = {f[1] * c->up[2] - f[2] * c->up[1], f[2] * c->up[0] - f[0] * c->up[2],
                 f[0] * c->up[1] - f[1] * c->up[0]};
  double rn = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  for (double &v : r) v /= rn;
  double u[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]};
  double th = std::tan(0.5 * (double)c->fov_y_deg * M_PI / 180.0);
  double aspect = (double)c->width / (double)c->height;
  for (int a = 0; a < 3; ++a) {
    j.eye[a] = (float)e[a];
    j.fwd[a] = (float)f[a];
    j.right[a] = (float)(r[a] * th * aspect);
    j.up[a] = (float)(u[a] * th);
  }
  j.width = c->width;
  j.height = c->height;
  j.spp = p->spp;
  j.max_steps = p->max_steps;
  j.stride = p->field_stride;
  j.light_mask = p->light_mask == 0 ? 0xF : p->light_mask;
  j.slot = p->field_slot;
  j.step = p->step_voxels / (float)ctx->nmax;
  j.t_min = p->t_min;
  j.g = p->g;
  j.inv_spp = 1.0f / (float)p->spp;
  j.seed = p->seed;
  j.out = out;
  j.bin0 = j.bin1 = 0;
  j.wbin = 0.0f;
  if (p->indirect == PFN_INDIRECT_CACHE) {
    int nb = ctx->cache_bins;
    double g = p->g;
    if (nb == 1 || g <= ctx->g_bins[0]) {
      j.bin0 = j.bin1 = 0;
    } else if (g >= ctx->g_bins[nb - 1]) {
      j.bin0 = j.bin1 = nb - 1;
    } else {
      int b = 0;
      while (b + 1 < nb - 1 && g >= ctx->g_bins[b + 1]) ++b;
      j.bin0 = b;
      j.bin1 = b + 1;
      j.wbin = (float)((g - ctx->g_bins[b]) / ((double)ctx->g_bins[b + 1] - ctx->g_bins[b]));
    }
  }
  const int bw = tc.tile_w * tc.block_w;
  j.blocks_x = (c->width + bw - 1) / bw;
  j.tiles_x = (c->width + tc.tile_w - 1) / tc.tile_w;
  j.tiles = j.tiles_x * ((c->height + tc.tile_h - 1) / tc.tile_h);
  j.ray_begin = 0;
}

pfn_status run_march(pfn_context *ctx, const pfn_render_job *jobs, int n_jobs, const TileConfig &tc,
                     bool first_interaction) {
  const pfn_render_params &p0 = jobs[0].params;
  std::vector<MarchJob> mj(n_jobs);
  int total = 0;
  for (int i = 0; i < n_jobs; ++i) {
    fill_job(ctx, &jobs[i].cam, &jobs[i].params, jobs[i].dev_rgb_out, tc, mj[i]);
    int bh = tc.tile_h * tc.block_h;
    int by = (jobs[i].cam.height + bh - 1) / bh;
    mj[i].block_begin = total;
    total += mj[i].blocks_x * by;
  }
  int prec = prec_of(p0.field_precision);
  std::vector<FieldDev> fd(PFN_MAX_FIELDS);
  std::vector<const void *> mp(PFN_MAX_FIELDS, nullptr);
  int mlp_bytes = 0;
  if (p0.indirect == PFN_INDIRECT_FIELD) {
    for (int s = 0; s < PFN_MAX_FIELDS; ++s) {
      FieldSlot &f = ctx->fields[s];
      if (!f.init) continue;
      bool used = false;
      for (int i = 0; i < n_jobs; ++i) used |= jobs[i].params.field_slot == s;
      if (!used) continue;
      pfn_status st = field_refresh(ctx, f, prec);
      if (st) return st;
      fd[s] = make_field_dev(f, prec);
      mp[s] = f.mlp_packed[prec];
      mlp_bytes = mlp_packed_elems(prec, f.desc.hidden_layers, f.desc.feats_per_level / 2) *
                  (prec == P_F32 ? 4 : 2);
    }
    for (int i = 0; i < n_jobs; ++i) {
      const pfn_field_desc &di = ctx->fields[jobs[i].params.field_slot].desc;
      const pfn_field_desc &d0 = ctx->fields[jobs[0].params.field_slot].desc;
      if (di.hidden_layers != d0.hidden_layers || di.feats_per_level != d0.feats_per_level)
        return pfn_fail(ctx, PFN_ERR_UNSUPPORTED,
                        "batched fields must share hidden_layers and feats_per_level");
    }
  }
  const bool wide_field = p0.indirect == PFN_INDIRECT_FIELD &&
                          ctx->fields[p0.field_slot].desc.feats_per_level != 2;
  // upload job table and field descriptors
  size_t jb = sizeof(MarchJob) * n_jobs;
  if (ctx->jobs_cap < (size_t)n_jobs) {
    dev_free(ctx->jobs_dev);
    PFN_HIP(ctx, dev_alloc((void **)&ctx->jobs_dev, jb));
    ctx->jobs_cap = n_jobs;
  }
  if (!ctx->fields_dev) {
    PFN_HIP(ctx, dev_alloc((void **)&ctx->fields_dev, sizeof(FieldDev) * PFN_MAX_FIELDS));
    PFN_HIP(ctx, dev_alloc((void **)&ctx->mlp_ptrs_dev, sizeof(void *) * PFN_MAX_FIELDS));
  }
  PFN_HIP(ctx, hipMemcpyAsync(ctx->jobs_dev, mj.data(), jb, hipMemcpyHostToDevice, ctx->stream));
  PFN_HIP(ctx, hipMemcpyAsync(ctx->fields_dev, fd.data(), sizeof(FieldDev) * PFN_MAX_FIELDS,
                              hipMemcpyHostToDevice, ctx->stream));
  PFN_HIP(ctx, hipMemcpyAsync(ctx->mlp_ptrs_dev, mp.data(), sizeof(void *) * PFN_MAX_FIELDS,
                              hipMemcpyHostToDevice, ctx->stream));
  PFN_HIP(ctx, hipStreamSynchronize(ctx->stream));  // host vectors go out of scope

  MarchArgs a{};
  a.vol = ctx->vol;
  a.vg = ctx->vol_grid;
  a.qvol = ctx->vol_dtype == PFN_F16 ? ctx->qvol : nullptr;
  a.qg = ctx->qvol_grid;
  a.tf = ctx->tf_dev;
  a.ext_scale = ctx->ext_scale;
  a.n_lights = ctx->n_lights;
  for (int l = 0; l < ctx->n_lights; ++l)
    for (int c = 0; c < 3; ++c) {
      a.light_pos[l][c] = ctx->lights[l].pos[c];
      a.light_int[l][c] = ctx->lights[l].intensity[c];
    }
  a.lightvol = ctx->lightvol;
  a.lvg = ctx->lv_grid;
  a.lquad = ctx->lv_valid && ctx->lquad_lights > 0 && ctx->lquad_lights == ctx->n_lights
                ? ctx->lquad
                : nullptr;
  a.lqg = ctx->lquad_grid;
  a.cache = ctx->cache;
  a.cache_res = ctx->cache_res;
  a.fields = ctx->fields_dev;
  a.mlp = (const void *const *)ctx->mlp_ptrs_dev;
  a.mlp_bytes = mlp_bytes;
  a.jobs = ctx->jobs_dev;
  a.n_jobs = n_jobs;
  a.total_blocks = total;
  a.tile_w = tc.tile_w;
  a.tile_h = tc.tile_h;
  a.block_w = tc.block_w;
  a.block_h = tc.block_h;
  a.counters = nullptr;
  a.persistent = tc.persistent;
  if (tc.persistent) {
    if (!ctx->queues) PFN_HIP(ctx, dev_alloc((void **)&ctx->queues, 64));
    a.queues = ctx->queues;
  }
  if (ctx->counting) {
    if (!ctx->counters) PFN_HIP(ctx, dev_alloc((void **)&ctx->counters, 16));
    PFN_HIP(ctx, hipMemsetAsync(ctx->counters, 0, 16, ctx->stream));
    a.counters = ctx->counters;
  }
  // the wavefront form when the caller (or the autotuner) chose it, or by default where no
  // graph replay was asked for; graph replay applies to the fused kernel only
  // (a field with 8 features per level is evaluated by the wavefront kernels only)
  const bool wavefront =
      p0.indirect == PFN_INDIRECT_FIELD &&
      (ctx->strategy == PFN_STRATEGY_WAVEFRONT || ctx->strategy == PFN_STRATEGY_WAVEFRONT_SERIAL ||
       (ctx->strategy == PFN_STRATEGY_AUTO && (!ctx->use_graph || wide_field)));
  if (wide_field && !wavefront && !first_interaction)
    return pfn_fail(ctx, PFN_ERR_UNSUPPORTED,
                    "the fused kernel evaluates fields of 2 features per level only");
  if (first_interaction) {
    pfn_status st = run_first_interaction(ctx, a, mj[0], p0.indirect, prec, p0.field_slot,
                                          fd[p0.field_slot]);
    if (st) return st;
  } else if (wavefront) {
    // wavefront rounds, one pass per field slot in use (the field kernel stages one slot's
    // weights); jobs keep their order within a pass
    std::vector<int> slots;
    for (int i = 0; i < n_jobs; ++i)
      if (std::find(slots.begin(), slots.end(), jobs[i].params.field_slot) == slots.end())
        slots.push_back(jobs[i].params.field_slot);
    for (int s : slots) {
      std::vector<MarchJob> part;
      for (int i = 0; i < n_jobs; ++i)
        if (jobs[i].params.field_slot == s) part.push_back(mj[i]);
      MarchArgs ap = a;
      ap.n_jobs = (int)part.size();
      pfn_status st = run_wavefront(ctx, ap, part, p0.direct, prec, s, fd[s],
                                    ctx->strategy != PFN_STRATEGY_WAVEFRONT_SERIAL);
      if (st) return st;
    }
  } else if (ctx->use_graph) {
    // replay a captured launch with the same arguments (the job table, field descriptors and
    // weight pointers it reads were refreshed above); capture it on first use
    std::vector<unsigned char> key(sizeof(MarchArgs) + 4 * sizeof(int));
    std::memcpy(key.data(), &a, sizeof(MarchArgs));
    int extra[4] = {(int)ctx->vol_dtype, p0.direct, p0.indirect, prec};
    std::memcpy(key.data() + sizeof(MarchArgs), extra, sizeof(extra));
    MarchGraph *g = nullptr;
    for (auto &e : ctx->graphs)
      if (e.key == key) g = &e;
    if (!g) {
      if (ctx->graphs.size() >= 16) {
        (void)hipGraphExecDestroy(ctx->graphs.front().exec);
        (void)hipGraphDestroy(ctx->graphs.front().graph);
        ctx->graphs.erase(ctx->graphs.begin());
      }
      if (!ctx->cap_stream)
        PFN_HIP(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
      MarchGraph ng;
      ng.key = key;
      PFN_HIP(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeRelaxed));
      hipError_t le = launch_march(a, ctx->vol_dtype, p0.direct, p0.indirect, prec, ctx->cap_stream);
      hipError_t ce = hipStreamEndCapture(ctx->cap_stream, &ng.graph);
      if (le != hipSuccess) return pfn_hip(ctx, le, "launch_march (capture)");
      if (ce != hipSuccess) return pfn_hip(ctx, ce, "hipStreamEndCapture");
      PFN_HIP(ctx, hipGraphInstantiate(&ng.exec, ng.graph, nullptr, nullptr, 0));
      ctx->graphs.push_back(ng);
      g = &ctx->graphs.back();
    }
    const int tslot = timing_begin(ctx);
    PFN_HIP(ctx, hipGraphLaunch(g->exec, ctx->stream));
    timing_end(ctx, tslot, TK_MARCH);
  } else {
    const int tslot = timing_begin(ctx);
    PFN_HIP(ctx, launch_march(a, ctx->vol_dtype, p0.direct, p0.indirect, prec, ctx->stream));
    timing_end(ctx, tslot, TK_MARCH);
  }
  if (ctx->counting) {
    PFN_HIP(ctx, hipMemcpyAsync(ctx->last_counts, ctx->counters, 16, hipMemcpyDeviceToHost,
                                ctx->stream));
    PFN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  }
  return PFN_OK;
}

extern "C" pfn_status pfn_render_frame(pfn_context *ctx, const pfn_camera *cam,
                                       const pfn_render_params *p, float *dev_rgb_out) {
  CHECK_CTX(ctx);
  pfn_status st = check_camera(ctx, cam);
  if (st) return st;
  st = check_render_params(ctx, p);
  if (st) return st;
  ARG(dev_rgb_out, "output is NULL");
  st = need_scene(ctx);
  if (st) return st;
  PFN_HIP(ctx, hipSetDevice(ctx->device));
  pfn_render_job job{*cam, *p, dev_rgb_out};
  return run_march(ctx, &job, 1, ctx->tile);
}

extern "C" pfn_status pfn_render_first_interaction(pfn_context *ctx, const pfn_camera *cam,
                                                   const pfn_render_params *p,
                                                   float *dev_rgb_out) {
  CHECK_CTX(ctx);
  pfn_status st = check_camera(ctx, cam);
  if (st) return st;
  ARG(p, "render params are NULL");
  pfn_render_params q = *p;
  q.direct = PFN_DIRECT_SHADOW_RAYS;  // direct light comes from delta-tracking visibility
  st = check_render_params(ctx, &q);
  if (st) return st;
  ARG(dev_rgb_out, "output is NULL");
  st = need_scene(ctx);
  if (st) return st;
  PFN_HIP(ctx, hipSetDevice(ctx->device));
  pfn_render_job job{*cam, q, dev_rgb_out};
  return run_march(ctx, &job, 1, ctx->tile, true);
}

extern "C" pfn_status pfn_render_batch(pfn_context *ctx, const pfn_render_job *jobs, int n_jobs) {
  CHECK_CTX(ctx);
  ARG(jobs && n_jobs >= 1 && n_jobs <= 4096, "1 to 4096 jobs");
  for (int i = 0; i < n_jobs; ++i) {
    pfn_status st = check_camera(ctx, &jobs[i].cam);
    if (st) return st;
    st = check_render_params(ctx, &jobs[i].params);
    if (st) return st;
    ARG(jobs[i].dev_rgb_out, "job output is NULL");
    ARG(jobs[i].params.indirect == jobs[0].params.indirect &&
            jobs[i].params.direct == jobs[0].params.direct &&
            jobs[i].params.field_precision == jobs[0].params.field_precision,
        "batched jobs must share indirect/direct mode and field precision");
  }
  pfn_status st = need_scene(ctx);
  if (st) return st;
  PFN_HIP(ctx, hipSetDevice(ctx->device));
  return run_march(ctx, jobs, n_jobs, ctx->tile);
}

// ------------------------------------------------------------------ photon map (Eq. 5)
extern "C" pfn_status pfn_photon_map_build(pfn_context *ctx, int grid_res) {
  CHECK_CTX(ctx);
  ARG(grid_res >= 1 && grid_res <= 128, "grid_res in [1, 128]");
  pfn_status st = need_scene(ctx);
  if (st) return st;
  if (ctx->rec_photons == 0) return pfn_fail(ctx, PFN_ERR_NOT_READY, "no trace yet");
  // the sorted map's offsets are 32-bit
  ARG(ctx->rec_count < ((uint64_t)1 << 32), "the photon map takes fewer than 2^32 records");
  PFN_HIP(ctx, hipSetDevice(ctx->device));
  PmSrcHost src{ctx->rec_x, ctx->rec_w, ctx->rec_p, ctx->rec_bin, ctx->rec_cnt, ctx->rec_maxrec,
                ctx->rec_photons * (uint64_t)ctx->rec_maxrec};
  return pm_build(ctx, src, ctx->cache_bins, ctx->g_bins, grid_res);
}

extern "C" pfn_status pfn_photon_map_set(pfn_context *ctx, const float *x, const float *w,
                                         const float *power, const int32_t *bin, uint64_t n,
                                         int n_bins, const float *g_bins, int grid_res) {
  CHECK_CTX(ctx);
  ARG(grid_res >= 1 && grid_res <= 128, "grid_res in [1, 128]");
  ARG(n_bins >= 1 && n_bins <= 8 && g_bins, "1 to 8 HG bins");
  ARG(n < ((uint64_t)1 << 32), "fewer than 2^32 records");
  ARG(n == 0 || (x && w && power && bin), "NULL record array");
  for (int i = 0; i < n_bins; ++i)
    ARG(std::isfinite(g_bins[i]) && std::fabs(g_bins[i]) <= 0.95f, "|g| <= 0.95");
  pfn_status st = need_scene(ctx);
  if (st) return st;
  PFN_HIP(ctx, hipSetDevice(ctx->device));
  PmSrcHost src{x, w, power, bin, nullptr, 1, n};
  return pm_build(ctx, src, n_bins, g_bins, grid_res);
}

extern "C" pfn_status pfn_photon_map_get(pfn_context *ctx, uint32_t *cell_start, size_t n_start,
                                         float *pos, float *dir, float *score, uint64_t capacity,
                                         uint64_t *host_n) {
  CHECK_CTX(ctx);
  if (!ctx->pmap.valid) return pfn_fail(ctx, PFN_ERR_NOT_READY, "no photon map");
  const PhotonMapState &m = ctx->pmap;
  const size_t keys = (size_t)m.n_bins * m.grid * m.grid * m.grid + 1;
  ARG(!cell_start || n_start == keys, "cell_start must hold n_bins * grid^3 + 1 entries");
  PFN_HIP(ctx, hipSetDevice(ctx->device));
  if (cell_start)
    PFN_HIP(ctx, hipMemcpyAsync(cell_start, m.start, keys * sizeof(uint32_t),
                                hipMemcpyDeviceToDevice, ctx->stream));
  const uint64_t n = std::min<uint64_t>(m.n, capacity);
  PFN_HIP(ctx, pm_launch_unpack(ctx, pos, dir, score, n));
  PFN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (host_n) *host_n = m.n;
  return PFN_OK;
}

extern "C" pfn_status pfn_photon_map_estimate(pfn_context *ctx, const float *xyz,
                                              const float *dir, const int32_t *bin, int64_t n,
                                              float radius, int k, float *rgb, float *r_out,
                                              int32_t *n_out) {
  CHECK_CTX(ctx);
  if (!ctx->pmap.valid) return pfn_fail(ctx, PFN_ERR_NOT_READY, "no photon map");
  ARG(n >= 0 && n < ((int64_t)1 << 31), "n in [0, 2^31)");
  ARG(n == 0 || (xyz && dir && bin && rgb), "NULL argument");
  ARG(std::isfinite(radius) && radius > 0.0f && radius <= 2.0f, "radius in (0, 2]");
  ARG(k >= 0 && k <= (1 << 20), "k in [0, 2^20]");
  PFN_HIP(ctx, hipSetDevice(ctx->device));
  const int tslot = timing_begin(ctx);
  PFN_HIP(ctx, pm_launch_estimate(ctx, xyz, dir, bin, n, radius, k, rgb, r_out, n_out,
                                  ctx->stream));
  timing_end(ctx, tslot, TK_PM_ESTIMATE);
  return PFN_OK;
}

// ------------------------------------------------------------------ timing
extern "C" pfn_status pfn_timing_enable(pfn_context *ctx, int on) {
  CHECK_CTX(ctx);
  ctx->timing = on != 0;
  return PFN_OK;
}

extern "C" pfn_status pfn_timing_get(pfn_context *ctx, int kernel, double *ms, int64_t *launches) {
  CHECK_CTX(ctx);
  ARG(kernel >= 0 && kernel < PFN_TIMED_KERNELS, "kernel id in [0, 16)");
  timing_collect(ctx);
  if (ms) *ms = ctx->t_ms[kernel];
  if (launches) *launches = ctx->t_n[kernel];
  return PFN_OK;
}

extern "C" pfn_status pfn_timing_reset(pfn_context *ctx) {
  CHECK_CTX(ctx);
  timing_collect(ctx);
  for (int i = 0; i < PFN_TIMED_KERNELS; ++i) {
    ctx->t_ms[i] = 0.0;
    ctx->t_n[i] = 0;
  }
  return PFN_OK;
}

extern "C" pfn_status pfn_set_render_strategy(pfn_context *ctx, int strategy) {
  CHECK_CTX(ctx);
  ARG(strategy == PFN_STRATEGY_AUTO || strategy == PFN_STRATEGY_FUSED ||
          strategy == PFN_STRATEGY_WAVEFRONT || strategy == PFN_STRATEGY_WAVEFRONT_SERIAL,
      "strategy is PFN_STRATEGY_AUTO, _FUSED, _WAVEFRONT or _WAVEFRONT_SERIAL");
  ctx->strategy = ctx->user_strategy = strategy;
  return PFN_OK;
}

extern "C" pfn_status pfn_set_tile_config(pfn_context *ctx, int tile_w, int block_w, int block_h) {
  CHECK_CTX(ctx);
  ARG(tile_w >= 1 && tile_w <= 64 && (tile_w & (tile_w - 1)) == 0,
      "tile_w in {1, 2, 4, 8, 16, 32, 64}");
  ARG(block_w >= 1 && block_h >= 1 && block_w * block_h == 4, "block_w * block_h must be 4");
  ctx->tile.tile_w = tile_w;
  ctx->tile.tile_h = 64 / tile_w;
  ctx->tile.block_w = block_w;
  ctx->tile.block_h = block_h;
  return PFN_OK;
}

extern "C" pfn_status pfn_set_launch_mode(pfn_context *ctx, int persistent_per_cu, int use_graph) {
  CHECK_CTX(ctx);
  ARG(persistent_per_cu >= 0 && persistent_per_cu <= 16, "persistent_per_cu in [0, 16]");
  ctx->tile.persistent = persistent_per_cu;
  ctx->use_graph = use_graph != 0;
  return PFN_OK;
}

// Time every candidate launch shape on the given batch and keep the fastest; results are cached
// per (batch shape, modes, volume) in the context.
extern "C" pfn_status pfn_autotune_batch(pfn_context *ctx, const pfn_render_job *jobs, int n_jobs,
                                         int iters, int *out_tile_w, int *out_block_w,
                                         int *out_block_h, int *out_persistent, int *out_strategy,
                                         double *out_ms) {
  CHECK_CTX(ctx);
  ARG(jobs && n_jobs >= 1 && n_jobs <= 4096, "1 to 4096 jobs");
  ARG(iters >= 1 && iters <= 100, "iters in [1, 100]");
  for (int i = 0; i < n_jobs; ++i) {
    pfn_status st = check_camera(ctx, &jobs[i].cam);
    if (st) return st;
    st = check_render_params(ctx, &jobs[i].params);
    if (st) return st;
    ARG(jobs[i].dev_rgb_out, "job output is NULL");
    ARG(jobs[i].params.indirect == jobs[0].params.indirect &&
            jobs[i].params.direct == jobs[0].params.direct &&
            jobs[i].params.field_precision == jobs[0].params.field_precision,
        "batched jobs must share indirect/direct mode and field precision");
  }
  pfn_status st = need_scene(ctx);
  if (st) return st;
  PFN_HIP(ctx, hipSetDevice(ctx->device));
  // cache key: job sizes and modes, volume shape; the render form is appended per form
  std::vector<unsigned char> base;
  auto put = [&base](const void *p, size_t n) {
    const unsigned char *c = (const unsigned char *)p;
    base.insert(base.end(), c, c + n);
  };
  for (int i = 0; i < n_jobs; ++i) {
    put(&jobs[i].cam.width, sizeof(int));
    put(&jobs[i].cam.height, sizeof(int));
    put(&jobs[i].params.spp, sizeof(int));
  }
  put(&jobs[0].params.indirect, sizeof(int));
  put(&jobs[0].params.direct, sizeof(int));
  put(&jobs[0].params.field_precision, sizeof(int));
  put(&ctx->vol_grid, sizeof(BrickGrid));
  put(&ctx->vol_dtype, sizeof(int));
  const bool field_lit = jobs[0].params.indirect == PFN_INDIRECT_FIELD;
  const int feats = field_lit ? ctx->fields[jobs[0].params.field_slot].desc.feats_per_level : 0;
  put(&feats, sizeof(int));
  // forms to time: the one the caller fixed, else the fused kernel (fields of 2 features per
  // level) and (field-lit batches) the overlapped wavefront rounds.  A form an earlier autotune
  // chose does not narrow them: the caller's setting decides.
  const int saved_strategy = ctx->strategy;
  std::vector<int> forms;
  if (ctx->user_strategy != PFN_STRATEGY_AUTO) forms.push_back(ctx->user_strategy);
  else {
    if (feats != 8) forms.push_back(PFN_STRATEGY_FUSED);
    if (field_lit) forms.push_back(PFN_STRATEGY_WAVEFRONT);
  }
  if (jobs[0].params.indirect != PFN_INDIRECT_FIELD) forms.assign(1, PFN_STRATEGY_FUSED);
  const bool saved_graph = ctx->use_graph, saved_timing = ctx->timing;
  TileConfig best{};
  double best_ms = -1.0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  // on every exit (errors included): the caller's launch settings back, the events freed
  struct Restore {
    pfn_context *c;
    bool graph, timing;
    int strategy;
    hipEvent_t *a, *b;
    ~Restore() {
      c->use_graph = graph;
      c->timing = timing;
      c->strategy = strategy;
      if (*a) (void)hipEventDestroy(*a);
      if (*b) (void)hipEventDestroy(*b);
    }
  } restore{ctx, saved_graph, saved_timing, saved_strategy, &e0, &e1};
  for (int form : forms) {
    std::vector<unsigned char> key = base;
    const int graph = form == PFN_STRATEGY_FUSED && saved_graph;
    key.insert(key.end(), (const unsigned char *)&form, (const unsigned char *)&form + sizeof(int));
    key.insert(key.end(), (const unsigned char *)&graph, (const unsigned char *)&graph + sizeof(int));
    const TunedEntry *hit = nullptr;
    for (const auto &e : ctx->tuned)
      if (e.key == key) hit = &e;
    TileConfig fbest{};
    double fms = -1.0;
    if (hit) {
      fbest = hit->best;
      fms = hit->ms;
    } else {
      if (!e0) {
        PFN_HIP(ctx, hipEventCreate(&e0));
        PFN_HIP(ctx, hipEventCreate(&e1));
      }
      // candidates: the fused kernel in every tile shape, block arrangement and launch mode;
      // the wavefront rounds in every tile shape (the march kernel's ray tiles)
      const int tws[4] = {4, 8, 16, 32};
      const int arr[3][2] = {{2, 2}, {4, 1}, {1, 4}};
      const int pers[3] = {0, 2, 4};
      std::vector<TileConfig> cands;
      for (int tw : tws) {
        TileConfig tc;
        tc.tile_w = tw;
        tc.tile_h = 64 / tw;
        tc.strategy = form;
        if (form != PFN_STRATEGY_FUSED) {
          cands.push_back(tc);
          continue;
        }
        for (auto &ar : arr)
          for (int pz : pers) {
            tc.block_w = ar[0];
            tc.block_h = ar[1];
            tc.persistent = pz;
            cands.push_back(tc);
          }
      }
      ctx->timing = false;
      ctx->strategy = form;
      ctx->use_graph = graph != 0;
      for (const TileConfig &tc : cands) {
        st = run_march(ctx, jobs, n_jobs, tc);  // warm-up (and graph capture)
        if (st) break;
        PFN_HIP(ctx, hipEventRecord(e0, ctx->stream));
        for (int it = 0; it < iters && !st; ++it) st = run_march(ctx, jobs, n_jobs, tc);
        PFN_HIP(ctx, hipEventRecord(e1, ctx->stream));
        PFN_HIP(ctx, hipEventSynchronize(e1));
        if (st) break;
        float ms = 0.0f;
        PFN_HIP(ctx, hipEventElapsedTime(&ms, e0, e1));
        const double per = ms / iters;
        if (fms < 0.0 || per < fms) {
          fms = per;
          fbest = tc;
        }
      }
      ctx->use_graph = saved_graph;
      ctx->timing = saved_timing;
      ctx->strategy = saved_strategy;
      if (st) break;
      ctx->tuned.push_back({key, fbest, fms});
    }
    if (best_ms < 0.0 || fms < best_ms) {
      best_ms = fms;
      best = fbest;
    }
  }
  if (st) return st;
  ctx->tile = best;
  restore.strategy = best.strategy;  // the chosen form becomes the context's (on return)
  if (out_strategy) *out_strategy = best.strategy;
  if (out_tile_w) *out_tile_w = best.tile_w;
  if (out_block_w) *out_block_w = best.block_w;
  if (out_block_h) *out_block_h = best.block_h;
  if (out_persistent) *out_persistent = best.persistent;
  if (out_ms) *out_ms = best_ms;
  return PFN_OK;
}

extern "C" pfn_status pfn_count_enable(pfn_context *ctx, int on) {
  CHECK_CTX(ctx);
  ctx->counting = on != 0;
  return PFN_OK;
}

extern "C" pfn_status pfn_count_get(pfn_context *ctx, uint64_t *steps, uint64_t *queries) {
  CHECK_CTX(ctx);
  if (steps) *steps = ctx->last_counts[0];
  if (queries) *queries = ctx->last_counts[1];
  return PFN_OK;
}
