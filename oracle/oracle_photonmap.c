/*
 * FP64 oracle, photon-map radiance estimate of Eq. (5) (test infrastructure only; see oracle.h).
 *
 * Over an explicit set of photon records (position, incident direction, incident power, HG bin):
 *  - each record's score is the collision estimator Phi / sigma_t(x_n) (the reading used for the
 *    isotropic cache as well, so that an isotropic phase function gives the cache's estimate);
 *  - the estimate at (x, w) for bin b takes the records of bin b around x and sums
 *    p_g(w_n . w) * score_n over them, divided by the sphere volume (4/3) pi r^3, with g the
 *    bin's anisotropy and w the direction of the scattered light (toward the viewer);
 *  - fixed radius: every record with |x_n - x| <= r;
 *  - KNN (Section 3.3): the K nearest records within the maximum radius r_max, and r the
 *    distance to the farthest of them (all of them if fewer than K lie within r_max; no record
 *    gives 0).
 * Brute force: every record is examined for every query.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle_internal.h"

void orc_pm_scores(const orc_scene *s, int64_t n, const double *x, const double *power,
                   double *score) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double sig, alb[3];
    orc_transfer(s, orc_density(s, x + 3 * i), &sig, alb);
    for (int c = 0; c < 3; ++c) score[3 * i + c] = sig > 0.0 ? power[3 * i + c] / sig : 0.0;
  }
}

typedef struct {
  double d2;
  int64_t idx;
} cand_t;

static int cand_cmp(const void *a, const void *b) {
  const cand_t *p = (const cand_t *)a, *q = (const cand_t *)b;
  if (p->d2 < q->d2) return -1;
  if (p->d2 > q->d2) return 1;
  return p->idx < q->idx ? -1 : (p->idx > q->idx ? 1 : 0);
}

void orc_pm_estimate(int64_t n_rec, const double *rx, const double *rw, const double *rs,
                     const int *rbin, const double *g_bins, double radius, int k, int64_t n_q,
                     const double *qx, const double *qw, const int *qbin, double *out,
                     double *r_used, int64_t *n_used) {
  const double r2max = radius * radius;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t q = 0; q < n_q; ++q) {
    const double *x = qx + 3 * q, *w = qw + 3 * q;
    const int b = qbin[q];
    const double g = g_bins[b];
    cand_t *cand = (cand_t *)malloc(sizeof(cand_t) * (size_t)(n_rec > 0 ? n_rec : 1));
    int64_t m = 0;
    for (int64_t i = 0; i < n_rec; ++i) {
      if (rbin[i] != b) continue;
      const double dx = rx[3 * i] - x[0], dy = rx[3 * i + 1] - x[1], dz = rx[3 * i + 2] - x[2];
      const double d2 = dx * dx + dy * dy + dz * dz;
      if (d2 <= r2max) {
        cand[m].d2 = d2;
        cand[m].idx = i;
        ++m;
      }
    }
    double r = radius;
    if (k > 0) {
      qsort(cand, (size_t)m, sizeof(cand_t), cand_cmp);
      if (m > k) m = k;
      r = m > 0 ? sqrt(cand[m - 1].d2) : 0.0;
    }
    double acc[3] = {0, 0, 0};
    for (int64_t j = 0; j < m; ++j) {
      const int64_t i = cand[j].idx;
      const double mu = rw[3 * i] * w[0] + rw[3 * i + 1] * w[1] + rw[3 * i + 2] * w[2];
      const double p = orc_hg_eval(g, mu);
      for (int c = 0; c < 3; ++c) acc[c] += p * rs[3 * i + c];
    }
    const double vol = 4.0 / 3.0 * M_PI * r * r * r;
    for (int c = 0; c < 3; ++c) out[3 * q + c] = (m > 0 && vol > 0.0) ? acc[c] / vol : 0.0;
    if (r_used) r_used[q] = (k > 0 && m == 0) ? 0.0 : r;
    if (n_used) n_used[q] = m;
    free(cand);
  }
}
