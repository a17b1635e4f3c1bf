/*
 * FP64 oracle, multi-phase photon tracing and the isotropic photon cache
 * (test infrastructure only; see oracle.h).
 *
 * Algorithm 1 (multi-phase photon tracing in heterogeneous media), read as follows:
 *  - photons are split equally over the lights and the phase pool (Section 4.4): photon `id`
 *    belongs to light id mod |L| and HG bin (id / |L|) mod |G|; its power is 4*pi*I divided by
 *    the number of photons of that (light, bin) pair;
 *  - emission from the point light is uniform over the cone of directions that contains the
 *    cube's bounding sphere, with the photon power scaled by the cone's share of the sphere
 *    (directions outside it never reach the volume, so this is the isotropic emission with the
 *    certain misses removed); free flights use delta tracking (Woodcock) with the global
 *    majorant ext_scale * max(A);
 *  - only interactions after the first are stored (Section 3.2), each with the power and
 *    direction with which the photon arrives there;
 *  - at a real collision the throughput is multiplied by the albedo (the opacity already sets
 *    the collision rate), then the direction is resampled from HG(g_bin);
 *  - the walk ends when the photon leaves the cube, after max_collisions real collisions, or by
 *    Russian roulette from collision rr_start on with survival probability min(1, max beta).
 * FP64 tallies account for every unit of emitted power.
 *
 * Cache: the collision estimator of fluence, Phi_n / sigma_t(x_n), splatted cloud-in-cell onto
 * the cell centres of a res^3 grid per bin and divided by 4*pi*V_cell, giving the direction
 * average of the in-scattered indirect radiance (the isotropic case of Eq. (5)).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include "oracle_internal.h"

typedef struct {
  double x[3], w[3], p[3];
  int bin;
} rec_t;

static void add3(double *dst, const double *v, double s) {
  for (int c = 0; c < 3; ++c) dst[c] += v[c] * s;
}

/* Trace one photon; records go to a caller buffer (at most max_collisions - 1 of them). */
static int trace_one(const orc_scene *s, const orc_trace_params *p, double majorant, uint64_t id,
                     orc_trace_stats *st, rec_t *recs) {
  int nL = s->n_lights, nB = p->n_bins;
  int l = (int)(id % (uint64_t)nL);
  int b = (int)((id / (uint64_t)nL) % (uint64_t)nB);
  uint64_t groups = (uint64_t)nL * (uint64_t)nB;
  uint64_t r = (uint64_t)l + (uint64_t)nL * (uint64_t)b;
  uint64_t n_lb = p->n_photons / groups + (r < p->n_photons % groups ? 1 : 0);
  const double *light = s->lights + 6 * l;
  orc_rng rng;
  orc_rng_init(&rng, p->seed, id, ORC_STREAM_TRACE);
  double u1 = orc_rng_next(&rng), u2 = orc_rng_next(&rng);
  double dir[3];
  double frac = orc_emit_dir(light, u1, u2, dir);
  double phi0[3];
  for (int c = 0; c < 3; ++c) phi0[c] = 4.0 * M_PI * frac * light[3 + c] / (double)n_lb;
  add3(st->emitted, phi0, 1.0);
  double o[3] = {light[0], light[1], light[2]};
  double t0, t1;
  if (!orc_clip_cube(o, dir, &t0, &t1)) {
    add3(st->escaped, phi0, 1.0);
    add3(st->escaped_uncollided, phi0, 1.0);
    return 0;
  }
  add3(st->entered, phi0, 1.0);
  double beta[3] = {1.0, 1.0, 1.0};
  double t = t0, tmax = t1;
  int coll = 0, nrec = 0;
  for (;;) {
    if (!(majorant > 0.0)) t = tmax;
    else t += -log(orc_rng_next(&rng)) / majorant;
    if (t >= tmax) {
      double pw[3] = {beta[0] * phi0[0], beta[1] * phi0[1], beta[2] * phi0[2]};
      add3(st->escaped, pw, 1.0);
      if (coll == 0) add3(st->escaped_uncollided, pw, 1.0);
      return nrec;
    }
    double x[3] = {o[0] + t * dir[0], o[1] + t * dir[1], o[2] + t * dir[2]};
    double sig, alb[3];
    orc_transfer(s, orc_density(s, x), &sig, alb);
    if (!(orc_rng_next(&rng) < sig / majorant)) {
      st->null_events += 1.0;
      continue;
    }
    coll += 1;
    st->collisions += 1.0;
    double pw[3] = {beta[0] * phi0[0], beta[1] * phi0[1], beta[2] * phi0[2]};
    if (coll >= 2) {
      rec_t *rc = &recs[nrec++];
      for (int a = 0; a < 3; ++a) {
        rc->x[a] = x[a];
        rc->w[a] = dir[a];
        rc->p[a] = pw[a];
      }
      rc->bin = b;
      add3(st->stored, pw, 1.0);
    }
    for (int c = 0; c < 3; ++c) st->absorbed[c] += pw[c] * (1.0 - alb[c]);
    for (int c = 0; c < 3; ++c) beta[c] *= alb[c];
    if (coll >= p->max_collisions) {
      for (int c = 0; c < 3; ++c) st->truncated[c] += beta[c] * phi0[c];
      return nrec;
    }
    double ua = orc_rng_next(&rng), ub = orc_rng_next(&rng);
    double nd[3];
    orc_hg_sample_dir(p->g_bins[b], dir, ua, ub, nd);
    dir[0] = nd[0];
    dir[1] = nd[1];
    dir[2] = nd[2];
    if (p->rr_start > 0 && coll >= p->rr_start) {
      double q = fmax(beta[0], fmax(beta[1], beta[2]));
      if (q > 1.0) q = 1.0;
      if (!(orc_rng_next(&rng) < q)) {
        for (int c = 0; c < 3; ++c) st->rr_killed[c] += beta[c] * phi0[c];
        return nrec;
      }
      for (int c = 0; c < 3; ++c) beta[c] /= q;
    }
    o[0] = x[0];
    o[1] = x[1];
    o[2] = x[2];
    t = 0.0;
    tmax = orc_exit_distance(o, dir);
  }
}

void orc_trace(const orc_scene *s, const orc_trace_params *p, uint64_t first, uint64_t count,
               orc_trace_stats *st_out, uint64_t cap, double *rec_x, double *rec_w, double *rec_pow,
               int *rec_bin, uint64_t *rec_photon, uint64_t *n_rec) {
  double majorant = orc_majorant(s);
  memset(st_out, 0, sizeof(*st_out));
  int maxrec = p->max_collisions > 1 ? p->max_collisions - 1 : 1;
  /* Per-photon record counts first (parallel), then an ordered copy. */
  rec_t *all = NULL;
  int *cnt = (int *)calloc(count ? count : 1, sizeof(int));
  int want = rec_x != NULL;
  if (want) all = (rec_t *)malloc((size_t)(count ? count : 1) * maxrec * sizeof(rec_t));
  int nthreads = orc_num_threads();
  orc_trace_stats *part = (orc_trace_stats *)calloc(nthreads, sizeof(orc_trace_stats));
#pragma omp parallel
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    rec_t local[64];
#pragma omp for schedule(dynamic, 256)
    for (uint64_t i = 0; i < count; ++i) {
      rec_t *dst = want ? all + i * (uint64_t)maxrec : local;
      cnt[i] = trace_one(s, p, majorant, first + i, &part[tid], dst);
    }
  }
  for (int t = 0; t < nthreads; ++t) {
    for (int c = 0; c < 3; ++c) {
      st_out->emitted[c] += part[t].emitted[c];
      st_out->entered[c] += part[t].entered[c];
      st_out->escaped[c] += part[t].escaped[c];
      st_out->escaped_uncollided[c] += part[t].escaped_uncollided[c];
      st_out->absorbed[c] += part[t].absorbed[c];
      st_out->truncated[c] += part[t].truncated[c];
      st_out->rr_killed[c] += part[t].rr_killed[c];
      st_out->stored[c] += part[t].stored[c];
    }
    st_out->collisions += part[t].collisions;
    st_out->null_events += part[t].null_events;
  }
  uint64_t total = 0;
  for (uint64_t i = 0; i < count; ++i) total += (uint64_t)cnt[i];
  st_out->n_records = total;
  uint64_t k = 0;
  if (want) {
    for (uint64_t i = 0; i < count; ++i)
      for (int j = 0; j < cnt[i]; ++j) {
        if (k >= cap) break;
        const rec_t *rc = all + i * (uint64_t)maxrec + j;
        for (int a = 0; a < 3; ++a) {
          rec_x[3 * k + a] = rc->x[a];
          rec_w[3 * k + a] = rc->w[a];
          rec_pow[3 * k + a] = rc->p[a];
        }
        rec_bin[k] = rc->bin;
        if (rec_photon) rec_photon[k] = first + i;
        ++k;
      }
  }
  if (n_rec) *n_rec = want ? k : total;
  free(part);
  free(cnt);
  free(all);
}

double orc_splat_cache(const orc_scene *s, int64_t n_rec, const double *rec_x, const double *rec_pow,
                       const int *rec_bin, int res, int n_bins, double *cache) {
  size_t cells = (size_t)res * res * res;
  memset(cache, 0, (size_t)n_bins * cells * 3 * sizeof(double));
  double norm = (double)cells / (4.0 * M_PI); /* 1 / (4 pi V_cell) */
  int n[3] = {res, res, res};
  for (int64_t k = 0; k < n_rec; ++k) {
    const double *x = rec_x + 3 * k;
    double sig, alb[3];
    orc_transfer(s, orc_density(s, x), &sig, alb);
    if (!(sig > 0.0)) continue;
    double xc[3];
    for (int a = 0; a < 3; ++a) xc[a] = fmin(1.0, fmax(0.0, x[a]));
    int i0[3], i1[3];
    double f[3];
    orc_cell_corners(xc, n, i0, i1, f);
    double *base = cache + (size_t)rec_bin[k] * cells * 3;
    for (int c = 0; c < 8; ++c) {
      int ix = (c & 1) ? i1[0] : i0[0];
      int iy = (c & 2) ? i1[1] : i0[1];
      int iz = (c & 4) ? i1[2] : i0[2];
      double w = ((c & 1) ? f[0] : 1.0 - f[0]) * ((c & 2) ? f[1] : 1.0 - f[1]) *
                 ((c & 4) ? f[2] : 1.0 - f[2]);
      double *e = base + (((size_t)iz * res + iy) * res + ix) * 3;
      for (int ch = 0; ch < 3; ++ch) e[ch] += w * rec_pow[3 * k + ch] / sig * norm;
    }
  }
  double kappa = 0.0;
  for (size_t i = 0; i < (size_t)n_bins * cells * 3; ++i)
    if (cache[i] > kappa) kappa = cache[i];
  return kappa;
}
