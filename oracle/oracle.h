/*
 * FP64 CPU oracle for Photon Field Networks (Bauer, Wu, Ma; arXiv 2304.07338).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that the
 * GPU path is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no source, header,
 * table or helper with the HIP library; both sides are written independently
 * from the paper and from the published definitions they cite.
 *
 * Everything is double precision.  Inputs that are random draws of the method
 * (photon emission, scattering, sub-pixel jitter, training batches) come from
 * Philox4x32-10 (Salmon et al., SC'11), implemented here from its published
 * definition.
 *
 * Geometry: the world is the unit cube [0,1]^3 (Section 3.1); every length and
 * every extinction coefficient is in cube units.
 */
#ifndef PFN_ORACLE_H
#define PFN_ORACLE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------- Counter-based RNG ---------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* uint32 -> (0,1): ((x >> 9) + 0.5) * 2^-23, exact in binary32 and binary64 */
double orc_u01(uint32_t x);
/* Fill n uniforms of stream (seed, item, stream_id) starting at draw 0. */
void orc_uniforms(uint64_t seed, uint64_t item, uint32_t stream_id, int n, double *out);

/* ---------------- Phase function (Section 3.2, Henyey-Greenstein) ---------------- */
double orc_hg_eval(double g, double mu);
double orc_hg_sample_mu(double g, double u);
void orc_hg_sample_dir(double g, const double w[3], double u1, double u2, double out[3]);

/* ---------------- Scene ---------------- */
typedef struct {
  const double *density; /* [nz][ny][nx], x fastest, values in [0,1] */
  int nx, ny, nz;
  const double *tf;      /* [256][4] RGBA; RGB = single-scattering albedo, A = opacity */
  double ext_scale;      /* sigma_t = ext_scale * A, per cube length */
  const double *lights;  /* [n_lights][6]: position xyz, radiant intensity rgb */
  int n_lights;
} orc_scene;

double orc_density(const orc_scene *s, const double x[3]);
void orc_transfer(const orc_scene *s, double rho, double *sigma_t, double albedo[3]);
double orc_majorant(const orc_scene *s);
int orc_clip_cube(const double o[3], const double d[3], double *t0, double *t1);
double orc_shadow_transmittance(const orc_scene *s, const double x[3], const double p[3],
                                double step);

/* ---------------- Photon cache (isotropic, per HG bin) ---------------- */
typedef struct {
  const double *data;  /* [n_bins][res^3][3], x fastest */
  int n_bins;
  const double *g_bins; /* ascending */
  int res;
} orc_cache;
void orc_cache_gather(const orc_cache *c, const double x[3], double g, double out[3]);

/* ---------------- Photon field (Sections 3.1, 3.3.2, 3.4) ---------------- */
typedef struct {
  int levels;        /* 16 */
  int feats;         /* features per level (2) */
  int base_res;      /* 16 */
  double growth;     /* 1.5 */
  int log2_table;    /* 19 */
  int hidden_layers; /* 3 */
  int width;         /* 64 */
  double psi;        /* 5 */
} orc_field_desc;

typedef struct {
  size_t pos_off[33], dir_off[33]; /* per-level entry offsets (in entries), [levels] = total */
  int pos_res[32], dir_res[32];
  int pos_dense[32], dir_dense[32];
  size_t pos_params, dir_params;   /* number of floats */
  size_t mlp_off;                  /* float offset of the first weight matrix */
  size_t w_off[8];                 /* float offset of each weight matrix */
  int w_rows[8], w_cols[8];
  int n_mats;
  int n_in;                        /* network input width */
  size_t n_params;
} orc_field_layout;

int orc_field_make_layout(const orc_field_desc *d, orc_field_layout *L);
size_t orc_field_num_params(const orc_field_desc *d);
/* rounding of parameters before use: 0 none, 1 binary16 RNE, 2 bfloat16 RNE */
void orc_field_forward(const orc_field_desc *d, const double *params, int rounding, int64_t n,
                       const double *xyz, const double *dir, const double *g, double *out_lp);
double orc_field_loss_grad(const orc_field_desc *d, const double *params, int rounding, int64_t n,
                           const double *xyz, const double *dir, const double *g,
                           const double *target, double *grad /* n_params, overwritten */);
/* The same with a choice of loss: 0 = L2, 1 = relative L2 (y - t)^2 / (y^2 + 0.01) per output,
 * the denominator held constant in the gradient. */
double orc_field_loss_grad_mode(const orc_field_desc *d, const double *params, int rounding,
                                int loss_mode, int64_t n, const double *xyz, const double *dir,
                                const double *g, const double *target, double *grad);
/* Encoding of one input: z has layout.n_in entries. */
void orc_field_encode(const orc_field_desc *d, const double *params, int rounding, const double x[3],
                      const double w[3], double g, double *z);
double orc_round_half(double v);
double orc_round_bf16(double v);

/* Log target encoding, Eq. (6), and its inverse, Eq. (7). */
double orc_log_encode(double v, double psi);
double orc_exp_decode(double lp, double psi);

/* ---------------- Training (Section 3.5.1) ---------------- */
void orc_adam_step(int64_t n, double *param, const double *grad, double *m, double *v, int64_t t,
                   double lr, double beta1, double beta2, double eps);
double orc_lr_at(int64_t step, double lr0, double decay, int64_t start_step, int64_t interval);
void orc_train_batch(uint64_t seed, int64_t step, int64_t n, const orc_cache *cache, double kappa,
                     double psi, double *xyz, double *dir, double *g, int *bin, double *target);
/* g_mode 0: g from the phase pool (the paper's batches); 1: g uniform over [g_0, g_last] with the
 * target interpolated linearly in g between the neighbouring bins. */
void orc_train_batch_mode(uint64_t seed, int64_t step, int64_t n, const orc_cache *cache,
                          double kappa, double psi, int g_mode, double *xyz, double *dir,
                          double *g, int *bin, double *target);
/* Samples first .. first + n - 1 of the same batch, written to rows 0 .. n - 1. */
void orc_train_batch_range(uint64_t seed, int64_t step, int64_t first, int64_t n,
                           const orc_cache *cache, double kappa, double psi, int g_mode,
                           double *xyz, double *dir, double *g, int *bin, double *target);

/* ---------------- Photon tracing (Algorithm 1) ---------------- */
typedef struct {
  uint64_t n_photons;
  int n_bins;
  double g_bins[8];
  int max_collisions;   /* 8 */
  int rr_start;         /* first collision index at which Russian roulette runs; <=0 disables */
  uint64_t seed;
} orc_trace_params;

typedef struct {
  double emitted[3], entered[3], escaped[3], escaped_uncollided[3], absorbed[3], truncated[3],
      rr_killed[3], stored[3];
  double collisions;   /* total real collisions */
  double null_events;  /* total null collisions */
  uint64_t n_records;
} orc_trace_stats;

/* Trace photons [first, first+count).  Records (if rec_* != NULL) are written in photon order,
 * collision order; *n_rec returns how many were produced (capacity cap).  rec_photon gets the id. */
void orc_trace(const orc_scene *s, const orc_trace_params *p, uint64_t first, uint64_t count,
               orc_trace_stats *st, uint64_t cap, double *rec_x, double *rec_w, double *rec_pow,
               int *rec_bin, uint64_t *rec_photon, uint64_t *n_rec);

/* Splat records into an isotropic per-bin cache [n_bins][res^3][3]; returns kappa = max. */
double orc_splat_cache(const orc_scene *s, int64_t n_rec, const double *rec_x, const double *rec_pow,
                       const int *rec_bin, int res, int n_bins, double *cache_out);

/* ---------------- Ray marcher (Sections 3.1 and 3.6) ---------------- */
typedef struct {
  double eye[3], target[3], up[3];
  double fov_y_deg;
  int width, height;
} orc_camera;

enum { ORC_IND_NONE = 0, ORC_IND_CACHE = 1, ORC_IND_FIELD = 2 };
enum { ORC_DIR_SHADOW = 0, ORC_DIR_LIGHTVOL = 1 };

typedef struct {
  int spp;
  double step_voxels;
  int max_steps;
  double t_min;
  int field_stride;
  double g;
  int indirect;
  int direct;
  int light_mask;   /* bit l set -> light l contributes; 0 = all lights */
  double lv_step_voxels; /* march step used to build the light transmittance grid */
  uint64_t seed;
} orc_render_params;

typedef struct {
  const orc_field_desc *desc;
  const double *params;
  int rounding;
  double kappa;
} orc_field;

void orc_camera_ray(const orc_camera *c, double px, double py, double o[3], double d[3]);
/* Render selected pixels (indices into the row-major width*height image); out is [n_pix][3]. */
void orc_render_pixels(const orc_scene *s, const orc_camera *c, const orc_render_params *p,
                       const orc_cache *cache, const orc_field *field, int64_t n_pix,
                       const int64_t *pix, double *out);
/* Light transmittance grid value at grid point (i,j,k) of a res^3 grid, light l. */
double orc_lightvol_point(const orc_scene *s, int res, int l, int i, int j, int k, double step);
int orc_lightvol_res(int n);

/* ---------------- Path tracer (Section 4.3 baseline) ---------------- */
void orc_pt_pixels(const orc_scene *s, const orc_camera *c, int spp, int max_bounces, double g,
                   int rr_start, uint64_t seed, int light_mask, int64_t n_pix, const int64_t *pix,
                   double *out);

/* ---------------- First-interaction renderer (Section 3.6, Algorithm 2) ---------------- */
/* One view ray per pixel through the pixel centre.  Each of its spp samples is an independent
 * delta-tracking walk (global majorant) from the cube entry to the first real collision; a
 * walk that leaves the cube is an invalid sample.  At a collision x with single-scattering
 * albedo a(x): L_d = sum_l I_l p_g(mu_l) V_l / r_l^2 with V_l in {0, 1} from a delta-tracking
 * walk toward light l, and L_i from the photon field (Eq. 2, decoded with Eq. 7) or the photon
 * cache.  The sample contributes a(x) * (L_d + L_i); the pixel is the mean over its spp samples.
 * Random numbers: the walk of sample s of pixel p uses Philox item p*spp + s of stream 10,
 * and the visibility walks from its collision item p*spp + s of stream 11 (lights in order,
 * one stream). */
typedef struct {
  int spp;
  double g;
  int indirect;     /* ORC_IND_NONE / ORC_IND_CACHE / ORC_IND_FIELD */
  int light_mask;   /* bit l set -> light l contributes; 0 = all lights */
  uint64_t seed;
} orc_fi_params;

/* Per sample, pixel-major ([n_pix][spp]): valid (1 = a collision), x[3], albedo[3], L_d[3] and
 * L_i[3] (zero for invalid samples).  Any output may be NULL. */
void orc_fi_samples(const orc_scene *s, const orc_camera *c, const orc_fi_params *p,
                    const orc_cache *cache, const orc_field *field, int64_t n_pix,
                    const int64_t *pix, int *valid, double *x, double *albedo, double *Ld,
                    double *Li);
/* Pixel values ([n_pix][3]). */
void orc_fi_pixels(const orc_scene *s, const orc_camera *c, const orc_fi_params *p,
                   const orc_cache *cache, const orc_field *field, int64_t n_pix,
                   const int64_t *pix, double *out);

/* ---------------- Photon-map radiance estimate (Eq. 5, Section 3.3) ---------------- */
/* Collision-estimator score Phi / sigma_t(x) of n records ([n][3] each). */
void orc_pm_scores(const orc_scene *s, int64_t n, const double *x, const double *power,
                   double *score);
/* Eq. (5) at n_q queries (position [3], unit direction of the scattered light [3], bin) over
 * n_rec records (position, incident direction, score, bin), brute force.  k = 0: every record of
 * the bin within `radius`, divided by the volume of that sphere; k > 0: the k nearest within
 * `radius`, divided by the sphere through the farthest of them.  out [n_q][3]; r_used and n_used
 * (may be NULL) receive the radius and the record count of each estimate. */
void orc_pm_estimate(int64_t n_rec, const double *rx, const double *rw, const double *rs,
                     const int *rbin, const double *g_bins, double radius, int k, int64_t n_q,
                     const double *qx, const double *qw, const int *qbin, double *out,
                     double *r_used, int64_t *n_used);

/* ---------------- Metrics ---------------- */
void orc_image_error(int64_t n, const double *img, const double *ref, double *rmse, double *rel_rmse,
                     double *psnr);

int orc_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
