/*
 * pfn.h — C ABI of the MI355X (gfx950) photon-field library.
 *
 * Photon Field Networks (Bauer, Wu, Ma; arXiv 2304.07338): a learned field P(x, g, w) -> RGB
 * (Eq. 2) that stands for the indirect in-scattered radiance L_i of Eq. (3)/(4), trained on
 * multi-phase photon caches (Section 3.2, Algorithm 1) and queried by a renderer that adds it to
 * direct light (Section 3.6).  The three top-level calls follow the paper's pipeline figure:
 * trace a multi-phase photon cache, train the field, render frames (retrain when the transfer
 * function or the lights change).
 *
 * Conventions for every call:
 *  - Return value: PFN_OK (0) or a negative pfn_status.  On error, pfn_last_error() describes it;
 *    arguments are validated before anything is launched, so an INVALID_ARG call has no effect.
 *  - Pointers named dev_* are device pointers on the context's device, owned by the caller and
 *    only borrowed for the call (the library never frees them and keeps no reference after the
 *    call returns unless stated).  host_* pointers are host memory.
 *  - Work is enqueued on the context stream.  Calls that return host_* results synchronise that
 *    stream before returning; dev_* results are ready in stream order (or after pfn_sync).
 *  - The unit cube [0,1]^3 is the world; lengths and extinction are in cube units.  Density
 *    volumes are [nz][ny][nx] with x fastest; voxel (i,j,k) has its centre at ((i+.5)/nx, ...).
 *  - A context is bound to one device and one stream; it is not thread-safe.
 */
#ifndef PFN_H
#define PFN_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PFN_OK = 0,
  PFN_ERR_INVALID_ARG = -1,
  PFN_ERR_OUT_OF_MEMORY = -2,
  PFN_ERR_HIP = -3,
  PFN_ERR_NOT_READY = -4,   /* a prerequisite (volume, cache, field, ...) is missing */
  PFN_ERR_UNSUPPORTED = -5, /* e.g. uniform g with photon-map targets */
  PFN_ERR_NUMERIC = -6      /* NaN or Inf met (e.g. in the training loss) */
} pfn_status;

typedef enum { PFN_F32 = 0, PFN_F16 = 1, PFN_BF16 = 2 } pfn_dtype;

typedef struct pfn_context pfn_context;

/* ------------------------------------------------------------------ context */
/* Create a context on HIP device `device`.  `hip_stream` (a hipStream_t) is used for all work;
 * NULL selects the device's null stream (ordered with every blocking stream, e.g. PyTorch's
 * default stream). */
pfn_status pfn_create(int device, void *hip_stream, pfn_context **out);
/* Free every context-owned buffer (volume bricks, caches, records, fields, optimiser state). */
void pfn_destroy(pfn_context *ctx);
/* Text of the last error on this context; valid until the next call on it. */
const char *pfn_last_error(const pfn_context *ctx);
pfn_status pfn_sync(pfn_context *ctx);
/* Replace the stream used for subsequent work (NULL = the null stream); waits for the old one. */
pfn_status pfn_set_stream(pfn_context *ctx, void *hip_stream);

/* ------------------------------------------------------------------ scene */
/* Scalar volume (Algorithm 1: Volume(x,y,z)): dev_density holds nx*ny*nz values of `dtype`
 * (PFN_F32 or PFN_F16) in [0,1], x fastest, copied into a context-owned brick layout.  A
 * PFN_F16 volume also gets a context-owned copy holding the four (x, y) corners of every cell
 * (8 bytes per cell, about 4x the volume: 1.1 GB at 512^3) for the ray marcher's density
 * lookups.  Sizes 2..4096, with fewer than 2^31 brick elements (PFN_ERR_INVALID_ARG
 * otherwise).  dev_density is read by a kernel enqueued on the context's stream: it must stay
 * valid until that work has run (stream order). */
pfn_status pfn_set_volume(pfn_context *ctx, const void *dev_density, pfn_dtype dtype, int nx,
                          int ny, int nz);
/* Transfer function (Algorithm 1: TransferFunction(sample)): 256 RGBA entries sampled at
 * density e/255; RGB is the single-scattering albedo, A the opacity; extinction
 * sigma_t = extinction_scale * A per cube length.  Values must be finite; RGB, A in [0,1]. */
pfn_status pfn_set_transfer_function(pfn_context *ctx, const float *host_rgba_256x4,
                                     float extinction_scale);
typedef struct {
  float pos[3];       /* cube units */
  float intensity[3]; /* radiant intensity (power per steradian), RGB */
} pfn_point_light;
/* Point lights (1..4).  Replacing lights or the transfer function invalidates the light volume. */
pfn_status pfn_set_lights(pfn_context *ctx, const pfn_point_light *host_lights, int n_lights);
/* Light-transmittance grid for direct light (one channel per light) at half the volume
 * resolution per axis, each value the exact shadow-march transmittance from the grid point to
 * the light with `step_voxels` steps (global shadows, Section 4.3).  With at most 3 lights and
 * at most 2^24 texels a context-owned copy holding the four (x, y) corner texels of every cell
 * (24 bytes per cell) is also built, for the ray marcher's lookups.  For a binary16 volume the
 * first build after pfn_set_volume also makes a context-owned copy of the density holding every
 * cell's eight corners (16 bytes per cell, 8x the volume: 17.6 GB at 1024^3), kept for later
 * builds while the volume stays; where it does not fit, the march reads the volume itself
 * (slower; the texels agree to FP32 rounding of the sample positions). */
pfn_status pfn_build_light_volume(pfn_context *ctx, float step_voxels);
/* Copy the light-transmittance grid to dev_out: rx * ry * rz texels (r = (n + 1) / 2 of each
 * volume side), x fastest, 4 binary16 values per texel (channel l = light l; unused channels
 * 1).  n_texels must equal rx * ry * rz.  PFN_ERR_NOT_READY without a built grid. */
pfn_status pfn_get_light_volume(pfn_context *ctx, uint16_t *dev_out, size_t n_texels);

/* ------------------------------------------------------------------ 1. photon cache */
typedef struct {
  uint64_t n_photons;   /* photon paths; split evenly over lights and HG bins (Section 4.4) */
  int n_bins;           /* |G|, 1..8 */
  float g_bins[8];      /* the phase pool G, ascending, |g| <= 0.95 */
  int cache_res;        /* cache grid resolution per axis, 2..512 */
  int max_collisions;   /* real collisions per photon path, 1..64 */
  int rr_start;         /* Russian roulette from this collision on; <= 0 disables it */
  uint64_t seed;
} pfn_trace_params;

typedef struct {
  uint64_t n_records;          /* stored photon interactions (collisions 2..max) */
  uint64_t n_records_dropped;  /* beyond the record buffer (0 unless the cap was hit) */
  double emitted[3], entered[3], escaped[3], escaped_uncollided[3], absorbed[3], truncated[3],
      rr_killed[3], stored[3]; /* power tallies (FP64) */
  double collisions, null_events;
  double kappa;                /* max cache value: the normaliser of the log target encoding */
} pfn_trace_stats;

/* Multi-phase photon tracing (Algorithm 1) and the isotropic per-bin photon cache built from its
 * records: the collision estimator Phi/sigma_t splatted cloud-in-cell and divided by
 * 4*pi*V_cell.  Requires volume, transfer function and lights.  Synchronises. */
pfn_status pfn_trace_photon_cache(pfn_context *ctx, const pfn_trace_params *params,
                                  pfn_trace_stats *host_stats);
/* Copy up to `capacity` photon records of the last trace in photon order:
 * position xyz, incident direction xyz, incident power RGB (float x3 each), HG bin, photon id.
 * Any output pointer may be NULL.  *host_count receives the number copied.  Synchronises. */
pfn_status pfn_get_records(pfn_context *ctx, float *dev_x, float *dev_w, float *dev_power,
                           int32_t *dev_bin, int64_t *dev_photon, uint64_t capacity,
                           uint64_t *host_count);
/* Cache as [n_bins][res][res][res][3] float (x fastest). */
pfn_status pfn_get_cache(pfn_context *ctx, float *dev_out, size_t n_floats);
pfn_status pfn_set_cache(pfn_context *ctx, const float *dev_in, int n_bins,
                         const float *host_g_bins, int res, double kappa);
pfn_status pfn_cache_info(pfn_context *ctx, int *host_n_bins, int *host_res, double *host_kappa);

/* Photon map and the radiance estimate of Eq. (5) (Section 3.3).  The map holds photon records
 * counting-sorted by (HG bin, cell of a uniform grid_res^3 grid over the unit cube); each keeps
 * its position, incident direction and the collision-estimator score Phi / sigma_t(x) (RGB, the
 * same normalisation as the isotropic cache, so that g = 0 reproduces the cache's estimate with
 * a sphere kernel).  The map is a snapshot: later traces or scene changes do not alter it.
 * pfn_photon_map_build takes the records of the last trace (its HG bins); pfn_photon_map_set
 * takes n records from device arrays (positions in [0,1]^3, unit incident directions and
 * incident powers [n][3], bins in [0, n_bins); records with a bin outside that range are
 * skipped).  Both need the volume and transfer function (for sigma_t) and synchronise.
 * grid_res in [1, 128]; device memory: 36 B per record plus 4 B x (n_bins grid_res^3 + 1) plus
 * 4 B per source record while building.  The map holds fewer than 2^32 records: n < 2^32, and
 * pfn_photon_map_build refuses (PFN_ERR_INVALID_ARG) a trace that kept 2^32 or more. */
pfn_status pfn_photon_map_build(pfn_context *ctx, int grid_res);
pfn_status pfn_photon_map_set(pfn_context *ctx, const float *dev_x, const float *dev_w,
                              const float *dev_power, const int32_t *dev_bin, uint64_t n,
                              int n_bins, const float *host_g_bins, int grid_res);
/* Copies of the map: dev_cell_start (n_bins grid_res^3 + 1 entries: the first record of every
 * key (bin, z, y, x), x fastest, then the total) and up to `capacity` sorted records
 * (position, direction, score [n][3]); records of one cell are in no particular order.  Any
 * output may be NULL; *host_n receives the record count.  Synchronises. */
pfn_status pfn_photon_map_get(pfn_context *ctx, uint32_t *dev_cell_start, size_t n_start,
                              float *dev_pos, float *dev_dir, float *dev_score,
                              uint64_t capacity, uint64_t *host_n);
/* Eq. (5) at n queries (position [n][3], unit direction of the scattered light [n][3] (toward
 * the viewer, as for the field), HG bin [n]) over the map's records of the query's bin:
 *   L = sum_n p_g(w_n . w) score_n / ((4/3) pi r^3), g the bin's anisotropy;
 *   k = 0: every record within `radius`, r = radius;
 *   k > 0: the k nearest records within `radius` (K-nearest query with a maximum radius), r the
 *          distance to the farthest of them (all records within `radius` if there are at most
 *          k; none gives 0).
 * Writes rgb [n][3] and, if not NULL, r [n] and the record count [n].  More than 256 records at
 * one distance (to 2^-40 of the radius) at the K-th place are cut to 256.  radius in (0, 2];
 * n < 2^31 (one wavefront per query; more than 2^24 queries run as several launches). */
pfn_status pfn_photon_map_estimate(pfn_context *ctx, const float *dev_xyz, const float *dev_dir,
                                   const int32_t *dev_bin, int64_t n, float radius, int k,
                                   float *dev_rgb, float *dev_r, int32_t *dev_count);

/* ------------------------------------------------------------------ 2. photon field */
typedef struct {
  int levels;          /* grid levels (1..16) */
  int feats_per_level; /* 2 or 8 (Section 3.4: the paper's encoding stores 8); renders of a field
                          with 8 run in the wavefront form only (the fused kernel returns
                          PFN_ERR_UNSUPPORTED for them) */
  int base_res;        /* coarsest grid resolution (2..4096) */
  float growth;        /* per-level resolution factor in [1, 4]; N_l = floor(base_res * growth^l),
                          below 2^24 cells per axis (16 levels at growth 2 from 16 reach 2^19) */
  int log2_table;      /* hashed-level table size 2^log2_table (dense levels are exact) */
  int hidden_layers;   /* ReLU hidden layers (1..7) of width 64, no biases, linear output;
                          the training calls take 1..5 (PFN_ERR_UNSUPPORTED above) */
  int width;           /* 64 */
  float psi;           /* log target encoding precision (Eq. 6/7) */
} pfn_field_desc;

/* Select the field slot (0..7) that the field calls below act on; each slot holds its own
 * parameters, optimiser state and kappa.  Renders use the slot in their parameters. */
pfn_status pfn_field_select(pfn_context *ctx, int slot);
/* Initialise the selected slot: grid features U(-1e-4, 1e-4), weights Glorot-uniform. */
pfn_status pfn_field_init(pfn_context *ctx, const pfn_field_desc *desc, uint64_t seed);
pfn_status pfn_field_num_params(pfn_context *ctx, size_t *host_n);
/* Parameter vector (FP32 master copy): [position grid][direction grid][W_0]...[W_H], each grid
 * level's entries holding feats_per_level consecutive features, each W row-major (out x in). */
pfn_status pfn_field_get_params(pfn_context *ctx, float *dev_out, size_t n);
pfn_status pfn_field_set_params(pfn_context *ctx, const float *dev_in, size_t n);
pfn_status pfn_field_set_kappa(pfn_context *ctx, double kappa);
/* Field inference (Eq. 2) at n points: xyz in [0,1]^3, unit directions (the view direction
 * pointing back along the ray), g.  Writes the raw network output L' (n x 3) and, if dev_rgb is
 * not NULL, the decoded radiance kappa * 10^(-psi L') (Eq. 7).  precision: arithmetic of the
 * grid features and MLP (F32, F16 or BF16 matrix cores, FP32 accumulation).  n < 2^38; more
 * than 2^30 queries run as several launches. */
pfn_status pfn_field_query(pfn_context *ctx, pfn_dtype precision, const float *dev_xyz,
                           const float *dev_dir, const float *dev_g, int64_t n,
                           float *dev_lprime, float *dev_rgb);
/* Loss over n x 3 outputs and its gradient with respect to every parameter (same layout as the
 * parameter vector), FP32 accumulation.  loss_mode 0: L2, mean((L' - target)^2); 1: relative L2
 * (Section 3.5.1), mean((L' - target)^2 / (L'^2 + 0.01)) with the denominator held constant in
 * the gradient.  Synchronises. */
pfn_status pfn_field_forward_backward(pfn_context *ctx, pfn_dtype precision, const float *dev_xyz,
                                      const float *dev_dir, const float *dev_g,
                                      const float *dev_target, int64_t n, int loss_mode,
                                      double *host_loss, float *dev_grad);

typedef struct {
  int steps;            /* training steps */
  int log2_batch;       /* samples per step = 2^log2_batch (8..22) */
  float lr, beta1, beta2, eps;
  float decay;          /* lr *= decay at decay_start and every decay_interval steps after */
  int decay_start, decay_interval;
  pfn_dtype precision;  /* F16 or BF16 matrix cores, or F32 */
  uint64_t seed;
  int target;           /* 0: the photon cache (gather); 1: the photon map, Eq. (5) */
  int knn_k;            /* photon-map targets: K nearest (0: every record within the radius) */
  float radius;         /* photon-map targets: the final (maximum) query radius, cube units */
  int staggered;        /* photon-map targets: 1 = the staggered schedule of Section 3.5.2 */
  int loss;             /* 0: L2 (the configuration); 1: relative L2 (Section 3.5.1) */
  int g_sampling;       /* 0: g drawn from the phase pool (Section 3.5.1); 1: g uniform over
                           [g_0, g_last], target = the cache gather interpolated linearly in g
                           between the two neighbouring bins (cache targets, >= 2 bins) */
} pfn_train_params;

/* Section 3.5: each step draws a fresh batch (uniform x, uniform direction, g from the cache
 * bins, or with g_sampling = 1 uniform between the first and last bin), takes its targets, runs
 * forward, L2 loss, backward and Adam.  Targets are Eq. (6) of
 * value / kappa (kappa: the cache maximum), the value being
 *   target 0: the cache gather at x in the sample's bin;
 *   target 1: the photon-map estimate of Eq. (5) at (x, direction) in the sample's bin, with
 *     knn_k and the step's radius: `radius` throughout, or with `staggered` the radii
 *     radius * {1/8, 1/4, 1/2, 1} over steps [0, 36 %), [36 %, 63 %), [63 %, 90 %),
 *     [90 %, 100 %) (the proportions of the paper's Table 1); the map (pfn_photon_map_build or
 *     _set) must hold the cache's HG bins.
 * Requires a cache and an initialised field.  host_loss_history (steps floats) may be NULL.
 * Synchronises. */
pfn_status pfn_train_field(pfn_context *ctx, const pfn_train_params *params,
                           float *host_loss_history);
/* The photon-map query radius that pfn_train_field uses at `step` (the staggered schedule of
 * Section 3.5.2 and Table 1, or the final radius); host only, no context, no GPU.  Returns
 * PFN_ERR_INVALID_ARG for NULL pointers, steps < 1 or step outside [0, steps). */
pfn_status pfn_train_step_radius(const pfn_train_params *params, int step, float *host_radius);
/* The learning rate that pfn_train_field applies at `step` (Section 3.5.1): lr until
 * decay_start, then lr * decay^(1 + floor((step - decay_start) / decay_interval)); with the
 * defaults (9e-4, 0.92, 1400, 25 over 2000 steps) the rate drops at 70 % of the run and every
 * 25 steps after.  Evaluated in FP64 and rounded to FP32 once, as the Adam launch receives it.
 * Host only, no context, no GPU.  Returns PFN_ERR_INVALID_ARG for NULL pointers, steps < 1,
 * step outside [0, steps), decay_interval < 1 or decay_start < 0. */
pfn_status pfn_train_lr_at(const pfn_train_params *params, int step, float *host_lr);
/* The training-batch generator alone (for checking): step `step`'s n samples, g_sampling as in
 * pfn_train_params (with one bin, 1 acts as 0).  dev_bin receives the sample's bin (uniform g:
 * the lower of the two neighbouring bins).  Any output may be NULL.  n in [0, 2^32] (sample i
 * draws from counter (step, i), so 2^32 samples are all distinct).  PFN_ERR_NOT_READY without a
 * cache. */
pfn_status pfn_train_batch(pfn_context *ctx, uint64_t seed, int64_t step, int64_t n,
                           int g_sampling, float *dev_xyz, float *dev_dir, float *dev_g,
                           int32_t *dev_bin, float *dev_target);
/* One Adam step (bias-corrected, step t >= 1) on the selected field with gradient dev_grad. */
pfn_status pfn_field_adam_step(pfn_context *ctx, const float *dev_grad, int64_t t, float lr,
                               float beta1, float beta2, float eps);

/* ------------------------------------------------------------------ 3. rendering */
typedef struct {
  float eye[3], target[3], up[3];
  float fov_y_deg;
  int width, height;
} pfn_camera;

typedef enum { PFN_INDIRECT_NONE = 0, PFN_INDIRECT_CACHE = 1, PFN_INDIRECT_FIELD = 2 } pfn_indirect;
typedef enum { PFN_DIRECT_SHADOW_RAYS = 0, PFN_DIRECT_LIGHT_VOLUME = 1 } pfn_direct;

typedef struct {
  int spp;              /* samples per pixel (1 = pixel centre, step midpoints) */
  float step_voxels;    /* march step in voxels of the largest volume dimension */
  int max_steps;        /* step cap per ray */
  float t_min;          /* stop when transmittance < t_min (0 = never) */
  int field_stride;     /* indirect light is evaluated every field_stride steps and held */
  float g;              /* HG anisotropy of the render, |g| <= 0.95 */
  pfn_indirect indirect;
  pfn_direct direct;
  pfn_dtype field_precision;
  int light_mask;       /* bit l selects light l; 0 = all lights */
  int field_slot;       /* field used when indirect = FIELD */
  uint64_t seed;        /* sub-pixel jitter when spp > 1 */
} pfn_render_params;

/* Ray-marched frame (Section 3.6 allows the field inside a ray marcher): per step the transfer
 * function, alpha = 1 - exp(-sigma_t l), direct in-scattered light from the point lights
 * (shadow rays or light volume), indirect in-scattered light from the field, the cache or none,
 * composited front to back: C += T alpha albedo (L_d + L_i); T *= exp(-sigma_t l).
 * Output dev_rgb_out: height x width x 3 floats (row 0 at the top). */
pfn_status pfn_render_frame(pfn_context *ctx, const pfn_camera *cam, const pfn_render_params *p,
                            float *dev_rgb_out);

typedef struct {
  pfn_camera cam;
  pfn_render_params params;
  float *dev_rgb_out;
} pfn_render_job;
/* Many frames of uneven sizes in one persistent launch (shared volume, per-job camera, lights,
 * g and field slot).  All jobs must share indirect/direct mode and field precision. */
pfn_status pfn_render_batch(pfn_context *ctx, const pfn_render_job *host_jobs, int n_jobs);

/* First-interaction renderer (Section 3.6, Algorithm 2).  One view ray per pixel through the
 * pixel centre; each of its spp samples is an independent delta-tracking walk (global majorant of
 * sigma_t) from the cube entry to the first real collision, and a walk that leaves the cube is an
 * invalid sample.  The collisions are compacted and the indirect light at all of them comes from
 * one batched pass of the field (or the photon cache, or none); the direct light is next-event
 * estimation toward every selected light with a delta-tracking visibility walk (V in {0, 1}).
 * Pixel = (1/spp) sum over valid samples of albedo * (L_d + L_i): a collision sampled in
 * proportion to sigma_t scatters with probability albedo = sigma_s / sigma_t, and the MIS
 * weights are 1 because point lights cannot be reached by phase sampling.
 * Uses spp, g, indirect, field_precision, light_mask, field_slot and seed of p (the march fields
 * and `direct` are ignored).  Random numbers: Philox item pixel * spp + s of stream 10 for the
 * walk of sample s; item pixel * spp + 16 j + k of stream 11 for the visibility walks of the k-th
 * collision among samples 16 j .. 16 j + 15.  Output dev_rgb_out: height x width x 3 floats.
 * Device buffers are those of the wavefront ray marcher (kept in the context); the direct-light
 * kernel runs on the library's second stream beside the field pass. */
pfn_status pfn_render_first_interaction(pfn_context *ctx, const pfn_camera *cam,
                                        const pfn_render_params *p, float *dev_rgb_out);

/* Monte Carlo volumetric path tracer (the baseline of Section 4.3): delta tracking, next-event
 * estimation with ratio tracking, HG sampling, at most max_bounces collisions. */
pfn_status pfn_render_path_traced(pfn_context *ctx, const pfn_camera *cam, int spp,
                                  int max_bounces, float g, int rr_start, int light_mask,
                                  uint64_t seed, float *dev_rgb_out);

/* RMSE, RMSE / mean(ref) and 20 log10(max(ref) / RMSE) over n floats, accumulated in FP64.
 * Synchronises. */
pfn_status pfn_image_error(pfn_context *ctx, const float *dev_img, const float *dev_ref, int64_t n,
                           double *host_rmse, double *host_rel_rmse, double *host_psnr);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * or evaluation loops, harnesses that forbid hipMalloc): the same three figures as
 * pfn_image_error, with no allocation of any kind and no synchronisation.  dev_result receives
 * (RMSE, RMSE / mean(ref), PSNR) as 3 doubles in device memory, ready in stream order.  The
 * FP64 partial sums live in a fixed device array of the library (64 KiB on each GPU it runs on,
 * held until the process ends): per-block partials, then one block adds them in a fixed order, so
 * results are bit-reproducible.  n is limited to 2048 * 256 * 64 = 33,554,432 values
 * (PFN_ERR_INVALID_ARG beyond, and for n < 1 or NULL pointers).  All calls on one GPU share the
 * array: calls that overlap on one GPU (other streams, contexts or threads) race. */
pfn_status pfn_image_error_noalloc(pfn_context *ctx, const float *dev_img, const float *dev_ref,
                                   int64_t n, double *dev_result);

/* Tile shape of the ray-march launch: each wave covers tile_w x (64 / tile_w) pixels (tile_w a
 * power of two, 1..64) and a workgroup block_w x block_h waves (block_w * block_h = 4).  Chosen
 * by the autotuner among tile_w 4, 8, 16 and 32. */
pfn_status pfn_set_tile_config(pfn_context *ctx, int tile_w, int block_w, int block_h);
/* Launch mode of the ray march: persistent_per_cu = 0 launches one workgroup per pixel block;
 * k > 0 launches k workgroups per compute unit that pull blocks from per-XCD queues until all
 * jobs are done.  use_graph != 0 captures each distinct launch into a HIP graph on first use and
 * replays it afterwards (the job table is refreshed before every replay). */
pfn_status pfn_set_launch_mode(pfn_context *ctx, int persistent_per_cu, int use_graph);
/* How field-lit frames are rendered (Section 3.6 ray marcher, both forms give the same pixels up
 * to the order of FP32 additions):
 *   PFN_STRATEGY_FUSED: one kernel marches, evaluates the field on the matrix cores inside the
 *     march loop and composites (the only form the persistent and graph launches use);
 *   PFN_STRATEGY_WAVEFRONT: rounds of a march kernel that stores up to 32 field queries per ray,
 *     level-major position-encoding kernels (each XCD encoding two levels, so that their
 *     tables stay in its L2) and a matrix-core field kernel per 16-query ray tile; a batch runs one pass
 *     of rounds per field slot it reads; never captured in graphs (the graph setting of
 *     pfn_set_launch_mode applies to the fused kernel only);
 *     the march kernel of the next round runs on the context's stream while this round's
 *     encoding kernels run on a second stream and its field kernel on a third (both owned by
 *     the library, default priority), beside the next round's encodings;
 *   PFN_STRATEGY_WAVEFRONT_SERIAL: the same rounds, all on the context's stream;
 *   PFN_STRATEGY_AUTO (default): the wavefront form, unless graph replay was asked for (then
 *     the fused kernel).
 * Device buffers of the wavefront form (two sets of about 2.9 KB per ray of a round with 16-bit
 * features, 5 KB with FP32, at most 2^21 rays per round, or 2^19 for fields of 8 features per
 * level, whose features take four times the room, plus 24 B per ray sample of the frame)
 * are kept in the context and grown on demand.  Both wavefront variants give bit-identical
 * images. */
typedef enum {
  PFN_STRATEGY_AUTO = 0,
  PFN_STRATEGY_FUSED = 1,
  PFN_STRATEGY_WAVEFRONT = 2,
  PFN_STRATEGY_WAVEFRONT_SERIAL = 3
} pfn_strategy;
pfn_status pfn_set_render_strategy(pfn_context *ctx, int strategy);
/* Autotuner: time on this batch (iters launches each, after one warm-up launch) the render
 * forms that the strategy last set by pfn_set_render_strategy allows (PFN_STRATEGY_AUTO, the
 * default: the fused kernel and, for field-lit batches, the overlapped wavefront rounds; any
 * other strategy: that form alone):
 *   - the fused kernel in every tile shape / block arrangement / launch mode, replayed from
 *     captured graphs if pfn_set_launch_mode asked for graphs;
 *   - the wavefront rounds in every tile shape.
 * It keeps the fastest for the context (tile shape, launch mode, and the render strategy, which
 * becomes that form until the next autotune or pfn_set_render_strategy; a later autotune again
 * tries every form the caller's strategy allows) and returns it.  Results are cached per batch shape and form (for the fused
 * kernel, also per graph setting).  host_strategy receives the chosen pfn_strategy; host_ms the
 * time of one launch of the batch in it; any output pointer may be NULL. */
pfn_status pfn_autotune_batch(pfn_context *ctx, const pfn_render_job *host_jobs, int n_jobs,
                              int iters, int *host_tile_w, int *host_block_w, int *host_block_h,
                              int *host_persistent, int *host_strategy, double *host_ms);

/* ------------------------------------------------------------------ timing */
/* When enabled, the main kernels are bracketed by HIP events on the stream they run on; the
 * accumulated device time (ms) and launch count per kernel are returned by pfn_timing_get.
 * kernel: 0 = ray march (a whole frame or batch, every kernel of it), 1 = photon trace,
 * 2 = training step (fused forward/backward), 3 = path tracer, 4 = field query, 5 = Adam;
 * kernels of the wavefront render: 6 = march rounds, 7 = position-encoding launches,
 * 8 = matrix-core field tiles, 9 = pixel resolve (the first-interaction renderer also reports
 * its field pass under 7 and 8 and its resolve under 9); first-interaction renderer:
 * 10 = ray generation, delta-tracking sampling and compaction, 11 = next-event estimation;
 * 12 = photon-map estimate; 13 = view-direction encoding of the wavefront and first-interaction
 * field passes.
 * Ids 0..15 are valid. */
pfn_status pfn_timing_enable(pfn_context *ctx, int on);
pfn_status pfn_timing_get(pfn_context *ctx, int kernel, double *host_ms, int64_t *host_launches);
pfn_status pfn_timing_reset(pfn_context *ctx);
/* When enabled, each ray-march launch also counts its march steps and its indirect-light
 * queries (field evaluations with non-zero weight, or cache gathers); the counts of the last
 * launch are returned by pfn_count_get.  Counting adds atomics and a synchronisation. */
pfn_status pfn_count_enable(pfn_context *ctx, int on);
pfn_status pfn_count_get(pfn_context *ctx, uint64_t *host_steps, uint64_t *host_queries);

#ifdef __cplusplus
}
#endif
#endif /* PFN_H */
