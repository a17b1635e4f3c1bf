/*
 * FP64 oracle, ray marcher and Monte Carlo path tracer (test infrastructure only; see oracle.h).
 *
 * Ray marcher (Section 3.6 allows the field to replace the multiple-scattering term of a ray
 * marcher; Eq. (3) splits the radiance into direct and indirect parts):
 *  - pinhole camera ray, clipped to the unit cube; black background;
 *  - fixed steps of step_voxels / max(nx,ny,nz) cube units, the last one clipped; sample at the
 *    midpoint of each step (or at the jitter offset xi when spp > 1);
 *  - per step: density, transfer function, alpha = 1 - exp(-sigma_t * l);
 *    direct in-scattered light L_d = sum_l I_l p_g(mu_l) T_l / r_l^2 (next-event estimation of
 *    Section 3.6, global shadows of Section 4.3), with T_l from an exact shadow march or from a
 *    light-transmittance grid at half the volume resolution;
 *    indirect in-scattered light L_i every `field_stride` steps (held in between) from the photon
 *    field (Eq. (2), decoded with Eq. (7)) or the photon cache;
 *    C += T * alpha * albedo * (L_d + L_i); T *= exp(-sigma_t * l); stop when T < t_min;
 *  - pixel = mean over spp samples (Composition, Section 3.6; MIS weights are 1 because point
 *    lights cannot be reached by phase sampling).
 *
 * Path tracer (the baseline of Section 4.3): delta tracking to real collisions, next-event
 * estimation with ratio tracking to every light, HG direction sampling, at most max_bounces
 * collisions, optional Russian roulette.
 *
 * First-interaction renderer (Section 3.6, Algorithm 2): ray generation, volume sampling by
 * delta tracking (several first interactions along one view ray), the indirect light from the
 * field at the interactions, direct light by next-event estimation with delta-tracking
 * visibility, and composition.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle_internal.h"

void orc_camera_ray(const orc_camera *c, double px, double py, double o[3], double d[3]) {
  double f[3] = {c->target[0] - c->eye[0], c->target[1] - c->eye[1], c->target[2] - c->eye[2]};
  orc_normalize(f);
  double r[3], u[3];
  orc_cross(f, c->up, r);
  orc_normalize(r);
  orc_cross(r, f, u);
  double th = tan(0.5 * c->fov_y_deg * M_PI / 180.0);
  double aspect = (double)c->width / (double)c->height;
  double sx = (2.0 * px / (double)c->width - 1.0) * th * aspect;
  double sy = (1.0 - 2.0 * py / (double)c->height) * th;
  for (int a = 0; a < 3; ++a) {
    o[a] = c->eye[a];
    d[a] = f[a] + sx * r[a] + sy * u[a];
  }
  orc_normalize(d);
}

int orc_lightvol_res(int n) { return (n + 1) / 2; }

double orc_lightvol_point(const orc_scene *s, int res, int l, int i, int j, int k, double step) {
  double x[3] = {((double)i + 0.5) / res, ((double)j + 0.5) / res, ((double)k + 0.5) / res};
  return orc_shadow_transmittance(s, x, s->lights + 6 * l, step);
}

typedef struct {
  int res[3];
  double step;
  double *memo; /* [n_lights][res^3], NaN = not computed yet */
} lightvol_t;

static double lightvol_value(const orc_scene *s, lightvol_t *lv, int l, int i, int j, int k) {
  size_t idx = (((size_t)l * lv->res[2] + k) * lv->res[1] + j) * lv->res[0] + i;
  double v;
#pragma omp atomic read
  v = lv->memo[idx];
  if (isnan(v)) {
    double x[3] = {((double)i + 0.5) / lv->res[0], ((double)j + 0.5) / lv->res[1],
                   ((double)k + 0.5) / lv->res[2]};
    v = orc_shadow_transmittance(s, x, s->lights + 6 * l, lv->step);
#pragma omp atomic write
    lv->memo[idx] = v;
  }
  return v;
}

static double lightvol_lookup(const orc_scene *s, lightvol_t *lv, int l, const double x[3]) {
  int i0[3], i1[3];
  double f[3];
  orc_cell_corners(x, lv->res, i0, i1, f);
  double acc = 0.0;
  for (int c = 0; c < 8; ++c) {
    int ix = (c & 1) ? i1[0] : i0[0];
    int iy = (c & 2) ? i1[1] : i0[1];
    int iz = (c & 4) ? i1[2] : i0[2];
    double w = ((c & 1) ? f[0] : 1.0 - f[0]) * ((c & 2) ? f[1] : 1.0 - f[1]) *
               ((c & 4) ? f[2] : 1.0 - f[2]);
    acc += w * lightvol_value(s, lv, l, ix, iy, iz);
  }
  return acc;
}

static int light_on(int mask, int l) { return mask == 0 || ((mask >> l) & 1); }

static void direct_light(const orc_scene *s, const orc_render_params *p, lightvol_t *lv,
                         const double x[3], const double wo[3], double step, double out[3]) {
  out[0] = out[1] = out[2] = 0.0;
  for (int l = 0; l < s->n_lights; ++l) {
    if (!light_on(p->light_mask, l)) continue;
    const double *L = s->lights + 6 * l;
    double v[3] = {x[0] - L[0], x[1] - L[1], x[2] - L[2]};
    double r2 = orc_dot(v, v);
    double r = sqrt(r2);
    double mu = orc_dot(v, wo) / r; /* light propagation direction . outgoing direction */
    double T = (p->direct == ORC_DIR_LIGHTVOL) ? lightvol_lookup(s, lv, l, x)
                                               : orc_shadow_transmittance(s, x, L, step);
    double k = orc_hg_eval(p->g, mu) * T / r2;
    for (int c = 0; c < 3; ++c) out[c] += L[3 + c] * k;
  }
}

typedef struct {
  orc_field_layout L;
} field_ctx;

static void indirect_light(const orc_render_params *p, const orc_cache *cache,
                           const orc_field *field, const double x[3], const double wo[3],
                           double out[3]) {
  out[0] = out[1] = out[2] = 0.0;
  if (p->indirect == ORC_IND_CACHE) {
    orc_cache_gather(cache, x, p->g, out);
  } else if (p->indirect == ORC_IND_FIELD) {
    double g = p->g, lp[3];
    /* orc_field_forward parallelises internally; one sample keeps it on this thread's work */
    orc_field_forward(field->desc, field->params, field->rounding, 1, x, wo, &g, lp);
    for (int c = 0; c < 3; ++c) out[c] = field->kappa * orc_exp_decode(lp[c], field->desc->psi);
  }
}

static void render_one(const orc_scene *s, const orc_camera *cam, const orc_render_params *p,
                       const orc_cache *cache, const orc_field *field, lightvol_t *lv, int64_t pix,
                       double out[3]) {
  int nmax = s->nx > s->ny ? s->nx : s->ny;
  if (s->nz > nmax) nmax = s->nz;
  double step = p->step_voxels / (double)nmax;
  int ix = (int)(pix % cam->width), iy = (int)(pix / cam->width);
  double acc[3] = {0, 0, 0};
  for (int smp = 0; smp < p->spp; ++smp) {
    double jx = 0.5, jy = 0.5, xi = 0.5;
    if (p->spp > 1) {
      orc_rng r;
      orc_rng_init(&r, p->seed, (uint64_t)pix * (uint64_t)p->spp + (uint64_t)smp,
                   ORC_STREAM_RENDER);
      jx = orc_rng_next(&r);
      jy = orc_rng_next(&r);
      xi = orc_rng_next(&r);
    }
    double o[3], d[3];
    orc_camera_ray(cam, (double)ix + jx, (double)iy + jy, o, d);
    double t0, t1;
    if (!orc_clip_cube(o, d, &t0, &t1)) continue;
    double span = t1 - t0;
    double nsteps = ceil(span / step);
    int64_t n = (int64_t)nsteps;
    if (n > p->max_steps) n = p->max_steps;
    double wo[3] = {-d[0], -d[1], -d[2]};
    double T = 1.0, C[3] = {0, 0, 0}, q[3] = {0, 0, 0};
    for (int64_t j = 0; j < n; ++j) {
      double l = fmin(step, span - (double)j * step);
      if (!(l > 0.0)) break;
      double t = t0 + (double)j * step + xi * l;
      double x[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
      double sig, alb[3];
      orc_transfer(s, orc_density(s, x), &sig, alb);
      double alpha = -expm1(-sig * l);
      double Ld[3];
      direct_light(s, p, lv, x, wo, step, Ld);
      if (j % p->field_stride == 0) indirect_light(p, cache, field, x, wo, q);
      for (int c = 0; c < 3; ++c) C[c] += T * alpha * alb[c] * (Ld[c] + q[c]);
      T *= exp(-sig * l);
      if (T < p->t_min) break;
    }
    for (int c = 0; c < 3; ++c) acc[c] += C[c];
  }
  for (int c = 0; c < 3; ++c) out[c] = acc[c] / (double)p->spp;
}

void orc_render_pixels(const orc_scene *s, const orc_camera *cam, const orc_render_params *p,
                       const orc_cache *cache, const orc_field *field, int64_t n_pix,
                       const int64_t *pix, double *out) {
  lightvol_t lv;
  memset(&lv, 0, sizeof(lv));
  if (p->direct == ORC_DIR_LIGHTVOL) {
    int nmax = s->nx > s->ny ? s->nx : s->ny;
    if (s->nz > nmax) nmax = s->nz;
    lv.res[0] = orc_lightvol_res(s->nx);
    lv.res[1] = orc_lightvol_res(s->ny);
    lv.res[2] = orc_lightvol_res(s->nz);
    lv.step = p->lv_step_voxels / (double)nmax;
    size_t cnt = (size_t)s->n_lights * lv.res[0] * lv.res[1] * lv.res[2];
    lv.memo = (double *)malloc(cnt * sizeof(double));
    for (size_t i = 0; i < cnt; ++i) lv.memo[i] = NAN;
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < n_pix; ++i) render_one(s, cam, p, cache, field, &lv, pix[i], out + 3 * i);
  free(lv.memo);
}

/* ------------------------------------------------------------------ path tracer */
static double ratio_tracking(const orc_scene *s, double majorant, const double x[3],
                             const double p[3], orc_rng *rng) {
  double v[3] = {p[0] - x[0], p[1] - x[1], p[2] - x[2]};
  double dist = sqrt(orc_dot(v, v));
  double d[3] = {v[0] / dist, v[1] / dist, v[2] / dist};
  double tmax = fmin(dist, orc_exit_distance(x, d));
  double T = 1.0, t = 0.0;
  if (!(majorant > 0.0)) return 1.0;
  for (;;) {
    t += -log(orc_rng_next(rng)) / majorant;
    if (t >= tmax) break;
    double xs[3] = {x[0] + t * d[0], x[1] + t * d[1], x[2] + t * d[2]};
    double sig, alb[3];
    orc_transfer(s, orc_density(s, xs), &sig, alb);
    T *= 1.0 - sig / majorant;
  }
  return T;
}

static void pt_one(const orc_scene *s, const orc_camera *cam, int spp, int max_bounces, double g,
                   int rr_start, uint64_t seed, int light_mask, double majorant, int64_t pix,
                   double out[3]) {
  int ix = (int)(pix % cam->width), iy = (int)(pix / cam->width);
  double acc[3] = {0, 0, 0};
  for (int smp = 0; smp < spp; ++smp) {
    orc_rng rng;
    orc_rng_init(&rng, seed, (uint64_t)pix * (uint64_t)spp + (uint64_t)smp, ORC_STREAM_PT);
    double jx = orc_rng_next(&rng), jy = orc_rng_next(&rng);
    double o[3], d[3];
    orc_camera_ray(cam, (double)ix + jx, (double)iy + jy, o, d);
    double t0, t1;
    if (!orc_clip_cube(o, d, &t0, &t1)) continue;
    double beta[3] = {1, 1, 1};
    double t = t0, tmax = t1;
    int k = 0;
    if (!(majorant > 0.0)) continue;
    for (;;) {
      t += -log(orc_rng_next(&rng)) / majorant;
      if (t >= tmax) break;
      double x[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
      double sig, alb[3];
      orc_transfer(s, orc_density(s, x), &sig, alb);
      if (!(orc_rng_next(&rng) < sig / majorant)) continue;
      k += 1;
      for (int l = 0; l < s->n_lights; ++l) {
        if (!light_on(light_mask, l)) continue;
        const double *L = s->lights + 6 * l;
        double v[3] = {x[0] - L[0], x[1] - L[1], x[2] - L[2]};
        double r2 = orc_dot(v, v);
        double mu = -orc_dot(v, d) / sqrt(r2);
        double T = ratio_tracking(s, majorant, x, L, &rng);
        double w = orc_hg_eval(g, mu) * T / r2;
        for (int c = 0; c < 3; ++c) acc[c] += beta[c] * alb[c] * L[3 + c] * w;
      }
      for (int c = 0; c < 3; ++c) beta[c] *= alb[c];
      if (k >= max_bounces) break;
      double ua = orc_rng_next(&rng), ub = orc_rng_next(&rng);
      double nd[3];
      orc_hg_sample_dir(g, d, ua, ub, nd);
      d[0] = nd[0];
      d[1] = nd[1];
      d[2] = nd[2];
      if (rr_start > 0 && k >= rr_start) {
        double q = fmin(1.0, fmax(beta[0], fmax(beta[1], beta[2])));
        if (!(orc_rng_next(&rng) < q)) break;
        for (int c = 0; c < 3; ++c) beta[c] /= q;
      }
      o[0] = x[0];
      o[1] = x[1];
      o[2] = x[2];
      t = 0.0;
      tmax = orc_exit_distance(o, d);
    }
  }
  for (int c = 0; c < 3; ++c) out[c] = acc[c] / (double)spp;
}

void orc_pt_pixels(const orc_scene *s, const orc_camera *cam, int spp, int max_bounces, double g,
                   int rr_start, uint64_t seed, int light_mask, int64_t n_pix, const int64_t *pix,
                   double *out) {
  double majorant = orc_majorant(s);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < n_pix; ++i)
    pt_one(s, cam, spp, max_bounces, g, rr_start, seed, light_mask, majorant, pix[i], out + 3 * i);
}

/* ------------------------------------------------------------------ first-interaction renderer */
/* Free-flight walk with the global majorant from x along unit d over [t, tmax): returns 1 and the
 * collision distance at the first real collision, 0 if the walk passes tmax. */
static int delta_track(const orc_scene *s, double majorant, const double x[3], const double d[3],
                       double t, double tmax, orc_rng *rng, double *t_hit) {
  if (!(majorant > 0.0)) return 0;
  for (;;) {
    t += -log(orc_rng_next(rng)) / majorant;
    if (t >= tmax) return 0;
    double xs[3] = {x[0] + t * d[0], x[1] + t * d[1], x[2] + t * d[2]};
    double sig, alb[3];
    orc_transfer(s, orc_density(s, xs), &sig, alb);
    if (orc_rng_next(rng) < sig / majorant) {
      *t_hit = t;
      return 1;
    }
  }
}

static void fi_one(const orc_scene *s, const orc_camera *cam, const orc_fi_params *p,
                   const orc_cache *cache, const orc_field *field, double majorant, int64_t pix,
                   int *valid, double *xo, double *albo, double *Ldo, double *Lio) {
  int ix = (int)(pix % cam->width), iy = (int)(pix / cam->width);
  double o[3], d[3];
  orc_camera_ray(cam, (double)ix + 0.5, (double)iy + 0.5, o, d);
  double t0 = 0.0, t1 = 0.0;
  const int hit = orc_clip_cube(o, d, &t0, &t1);
  const double wo[3] = {-d[0], -d[1], -d[2]};
  orc_render_params ip;
  memset(&ip, 0, sizeof(ip));
  ip.g = p->g;
  ip.indirect = p->indirect;
  for (int smp = 0; smp < p->spp; ++smp) {
    int ok = 0;
    double x[3] = {0, 0, 0}, alb[3] = {0, 0, 0}, Ld[3] = {0, 0, 0}, Li[3] = {0, 0, 0};
    if (hit) {
      /* Volume sampling: the first real collision of this sample's walk */
      orc_rng rng;
      orc_rng_init(&rng, p->seed, (uint64_t)pix * (uint64_t)p->spp + (uint64_t)smp,
                   ORC_STREAM_FI_SAMPLE);
      double th;
      ok = delta_track(s, majorant, o, d, t0, t1, &rng, &th);
      if (ok) {
        for (int c = 0; c < 3; ++c) x[c] = o[c] + th * d[c];
        double sig;
        orc_transfer(s, orc_density(s, x), &sig, alb);
        /* Direct illumination: next-event estimation, visibility by delta tracking */
        orc_rng vr;
        orc_rng_init(&vr, p->seed, (uint64_t)pix * (uint64_t)p->spp + (uint64_t)smp,
                     ORC_STREAM_FI_NEE);
        for (int l = 0; l < s->n_lights; ++l) {
          if (!light_on(p->light_mask, l)) continue;
          const double *L = s->lights + 6 * l;
          double v[3] = {x[0] - L[0], x[1] - L[1], x[2] - L[2]};
          double r2 = orc_dot(v, v);
          double r = sqrt(r2);
          double mu = orc_dot(v, wo) / r;
          double dl[3] = {-v[0] / r, -v[1] / r, -v[2] / r};
          double tmax = fmin(r, orc_exit_distance(x, dl));
          double tb;
          double V = delta_track(s, majorant, x, dl, 0.0, tmax, &vr, &tb) ? 0.0 : 1.0;
          double w = orc_hg_eval(p->g, mu) * V / r2;
          for (int c = 0; c < 3; ++c) Ld[c] += L[3 + c] * w;
        }
        /* Photon field prediction and decoding (or the cache) at the interaction */
        indirect_light(&ip, cache, field, x, wo, Li);
      }
    }
    const int64_t j = (int64_t)smp;
    if (valid) valid[j] = ok;
    for (int c = 0; c < 3; ++c) {
      if (xo) xo[3 * j + c] = x[c];
      if (albo) albo[3 * j + c] = alb[c];
      if (Ldo) Ldo[3 * j + c] = Ld[c];
      if (Lio) Lio[3 * j + c] = Li[c];
    }
  }
}

void orc_fi_samples(const orc_scene *s, const orc_camera *cam, const orc_fi_params *p,
                    const orc_cache *cache, const orc_field *field, int64_t n_pix,
                    const int64_t *pix, int *valid, double *x, double *albedo, double *Ld,
                    double *Li) {
  const double majorant = orc_majorant(s);
  const int64_t S = p->spp;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < n_pix; ++i)
    fi_one(s, cam, p, cache, field, majorant, pix[i], valid ? valid + i * S : NULL,
           x ? x + 3 * i * S : NULL, albedo ? albedo + 3 * i * S : NULL,
           Ld ? Ld + 3 * i * S : NULL, Li ? Li + 3 * i * S : NULL);
}

/* Composition: L = (1/spp) sum_k a_k (L_d,k + L_i,k); invalid samples contribute nothing. */
void orc_fi_pixels(const orc_scene *s, const orc_camera *cam, const orc_fi_params *p,
                   const orc_cache *cache, const orc_field *field, int64_t n_pix,
                   const int64_t *pix, double *out) {
  const int64_t S = p->spp;
  double *alb = (double *)malloc(sizeof(double) * 3 * S * (size_t)(n_pix > 0 ? n_pix : 1));
  double *Ld = (double *)malloc(sizeof(double) * 3 * S * (size_t)(n_pix > 0 ? n_pix : 1));
  double *Li = (double *)malloc(sizeof(double) * 3 * S * (size_t)(n_pix > 0 ? n_pix : 1));
  orc_fi_samples(s, cam, p, cache, field, n_pix, pix, NULL, NULL, alb, Ld, Li);
  for (int64_t i = 0; i < n_pix; ++i)
    for (int c = 0; c < 3; ++c) {
      double acc = 0.0;
      for (int64_t j = 0; j < S; ++j) {
        const size_t q = (size_t)(3 * (i * S + j) + c);
        acc += alb[q] * (Ld[q] + Li[q]);
      }
      out[3 * i + c] = acc / (double)S;
    }
  free(alb);
  free(Ld);
  free(Li);
}
