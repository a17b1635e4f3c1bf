/*
 * FP64 oracle, core definitions (test infrastructure only; see oracle.h).
 *
 *  - Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, "Parallel random
 *    numbers: as easy as 1, 2, 3", SC'11), written from its published definition.
 *  - Henyey-Greenstein phase function (Section 3.2 and its phase-function figure): the
 *    textbook density and inverse-CDF sampler.
 *  - Scalar volume, transfer function and optics (Algorithm 1: Volume(x,y,z) and
 *    TransferFunction(sample); Section 3.6 Composition: scattering from the albedo).
 *  - Photon-cache gather and the image error metrics (Section 4.3.2).
 */
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include "oracle_internal.h"

/* ------------------------------------------------------------------ Philox4x32-10 */
/* Multipliers and Weyl key increments as published with the algorithm. */
#define PHILOX_MUL0 0xD2511F53u
#define PHILOX_MUL1 0xCD9E8D57u
#define PHILOX_WEYL0 0x9E3779B9u
#define PHILOX_WEYL1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_WEYL0;
      k1 += PHILOX_WEYL1;
    }
    uint64_t p0 = (uint64_t)PHILOX_MUL0 * (uint64_t)c0;
    uint64_t p1 = (uint64_t)PHILOX_MUL1 * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

double orc_u01(uint32_t x) {
  /* 23 random bits, centred in their bucket: (k + 1/2) / 2^23, never 0 or 1. */
  return ((double)(x >> 9) + 0.5) * (1.0 / 8388608.0);
}

void orc_uniforms(uint64_t seed, uint64_t item, uint32_t stream_id, int n, double *out) {
  orc_rng r;
  orc_rng_init(&r, seed, item, stream_id);
  for (int i = 0; i < n; ++i) out[i] = orc_rng_next(&r);
}

/* ------------------------------------------------------------------ Henyey-Greenstein */
double orc_hg_eval(double g, double mu) {
  double denom = 1.0 + g * g - 2.0 * g * mu;
  return (1.0 - g * g) / (4.0 * M_PI * denom * sqrt(denom));
}

double orc_hg_sample_mu(double g, double u) {
  if (fabs(g) < 1e-3) return 1.0 - 2.0 * u;
  double sq = (1.0 - g * g) / (1.0 - g + 2.0 * g * u);
  double mu = (1.0 + g * g - sq * sq) / (2.0 * g);
  if (mu > 1.0) mu = 1.0;
  if (mu < -1.0) mu = -1.0;
  return mu;
}

/* Orthonormal basis around unit n, following Duff et al., "Building an Orthonormal Basis,
 * Revisited" (JCGT 2017). */
static void onb(const double n[3], double t1[3], double t2[3]) {
  double sign = n[2] >= 0.0 ? 1.0 : -1.0;
  double a = -1.0 / (sign + n[2]);
  double b = n[0] * n[1] * a;
  t1[0] = 1.0 + sign * n[0] * n[0] * a;
  t1[1] = sign * b;
  t1[2] = -sign * n[0];
  t2[0] = b;
  t2[1] = sign + n[1] * n[1] * a;
  t2[2] = -n[1];
}

void orc_hg_sample_dir(double g, const double w[3], double u1, double u2, double out[3]) {
  double mu = orc_hg_sample_mu(g, u1);
  double s = sqrt(fmax(0.0, 1.0 - mu * mu));
  double phi = 2.0 * M_PI * u2;
  double t1[3], t2[3];
  onb(w, t1, t2);
  double cp = cos(phi), sp = sin(phi);
  for (int a = 0; a < 3; ++a) out[a] = mu * w[a] + s * (cp * t1[a] + sp * t2[a]);
  orc_normalize(out);
}

/* Emission from a point light p: uniform over the cone around the direction to the cube centre
 * that just contains the cube's bounding sphere (radius sqrt(3)/2), or over the whole sphere
 * when the light lies inside that sphere.  Returns the solid-angle fraction of the emitted
 * directions (1 for the whole sphere), which scales the photon power so that the estimate stays
 * unbiased: directions outside the cone cannot reach the cube. */
double orc_emit_dir(const double p[3], double u1, double u2, double out[3]) {
  double c[3] = {0.5 - p[0], 0.5 - p[1], 0.5 - p[2]};
  double d = sqrt(orc_dot(c, c));
  const double R = 0.5 * sqrt(3.0);
  if (!(d > R)) {
    orc_iso_dir(u1, u2, out);
    return 1.0;
  }
  double axis[3] = {c[0] / d, c[1] / d, c[2] / d};
  double cos_a = sqrt(1.0 - (R / d) * (R / d));
  double ct = 1.0 - u1 * (1.0 - cos_a);
  double st = sqrt(fmax(0.0, 1.0 - ct * ct));
  double phi = 2.0 * M_PI * u2;
  double t1[3], t2[3];
  onb(axis, t1, t2);
  double cp = cos(phi), sp = sin(phi);
  for (int a = 0; a < 3; ++a) out[a] = ct * axis[a] + st * (cp * t1[a] + sp * t2[a]);
  orc_normalize(out);
  return 0.5 * (1.0 - cos_a);
}

void orc_iso_dir(double u1, double u2, double out[3]) {
  double z = 1.0 - 2.0 * u1;
  double r = sqrt(fmax(0.0, 1.0 - z * z));
  double phi = 2.0 * M_PI * u2;
  out[0] = r * cos(phi);
  out[1] = r * sin(phi);
  out[2] = z;
}

/* ------------------------------------------------------------------ volume and optics */
void orc_cell_corners(const double x[3], const int n[3], int i0[3], int i1[3], double f[3]) {
  for (int a = 0; a < 3; ++a) {
    double u = x[a] * (double)n[a] - 0.5;
    double fl = floor(u);
    f[a] = u - fl;
    int lo = (int)fl, hi = (int)fl + 1;
    if (lo < 0) lo = 0;
    if (lo > n[a] - 1) lo = n[a] - 1;
    if (hi < 0) hi = 0;
    if (hi > n[a] - 1) hi = n[a] - 1;
    i0[a] = lo;
    i1[a] = hi;
  }
}

double orc_density(const orc_scene *s, const double x[3]) {
  for (int a = 0; a < 3; ++a)
    if (!(x[a] >= 0.0 && x[a] <= 1.0)) return 0.0;
  int n[3] = {s->nx, s->ny, s->nz};
  int i0[3], i1[3];
  double f[3];
  orc_cell_corners(x, n, i0, i1, f);
  double acc = 0.0;
  for (int c = 0; c < 8; ++c) {
    int ix = (c & 1) ? i1[0] : i0[0];
    int iy = (c & 2) ? i1[1] : i0[1];
    int iz = (c & 4) ? i1[2] : i0[2];
    double w = ((c & 1) ? f[0] : 1.0 - f[0]) * ((c & 2) ? f[1] : 1.0 - f[1]) *
               ((c & 4) ? f[2] : 1.0 - f[2]);
    acc += w * s->density[((size_t)iz * s->ny + iy) * s->nx + ix];
  }
  return acc;
}

void orc_transfer(const orc_scene *s, double rho, double *sigma_t, double albedo[3]) {
  double u = rho * 255.0;
  if (u < 0.0) u = 0.0;
  if (u > 255.0) u = 255.0;
  int i = (int)floor(u);
  if (i > 254) i = 254;
  double f = u - (double)i;
  const double *a = s->tf + 4 * i, *b = s->tf + 4 * (i + 1);
  for (int c = 0; c < 3; ++c) albedo[c] = (1.0 - f) * a[c] + f * b[c];
  *sigma_t = s->ext_scale * ((1.0 - f) * a[3] + f * b[3]);
}

double orc_majorant(const orc_scene *s) {
  double m = 0.0;
  for (int i = 0; i < 256; ++i) m = fmax(m, s->tf[4 * i + 3]);
  return m * s->ext_scale;
}

int orc_clip_cube(const double o[3], const double d[3], double *t0, double *t1) {
  double tn = -DBL_MAX, tf = DBL_MAX;
  for (int a = 0; a < 3; ++a) {
    if (d[a] == 0.0) {
      if (o[a] < 0.0 || o[a] > 1.0) return 0;
      continue;
    }
    double ta = (0.0 - o[a]) / d[a];
    double tb = (1.0 - o[a]) / d[a];
    if (ta > tb) {
      double t = ta;
      ta = tb;
      tb = t;
    }
    if (ta > tn) tn = ta;
    if (tb < tf) tf = tb;
  }
  if (tn < 0.0) tn = 0.0;
  if (!(tn < tf)) return 0;
  *t0 = tn;
  *t1 = tf;
  return 1;
}

double orc_exit_distance(const double x[3], const double d[3]) {
  double t = DBL_MAX;
  for (int a = 0; a < 3; ++a) {
    if (d[a] > 0.0) t = fmin(t, (1.0 - x[a]) / d[a]);
    else if (d[a] < 0.0) t = fmin(t, (0.0 - x[a]) / d[a]);
  }
  return t < 0.0 ? 0.0 : t;
}

/* Transmittance from x to the point light at p: midpoint quadrature of the optical depth
 * with the march step, over the part of the segment inside the cube (global shadows,
 * Section 4.3; next-event estimation, Section 3.6). */
double orc_shadow_transmittance(const orc_scene *s, const double x[3], const double p[3],
                                double step) {
  double v[3] = {p[0] - x[0], p[1] - x[1], p[2] - x[2]};
  double dist = sqrt(orc_dot(v, v));
  if (dist <= 0.0) return 1.0;
  double d[3] = {v[0] / dist, v[1] / dist, v[2] / dist};
  double t0, t1;
  if (!orc_clip_cube(x, d, &t0, &t1)) return 1.0;
  double tend = fmin(t1, dist);
  if (!(tend > t0)) return 1.0;
  double len = tend - t0;
  double tau = 0.0;
  for (int64_t k = 0;; ++k) {
    double l = fmin(step, len - (double)k * step);
    if (!(l > 0.0)) break;
    double t = t0 + (double)k * step + 0.5 * l;
    double xs[3] = {x[0] + t * d[0], x[1] + t * d[1], x[2] + t * d[2]};
    double sig, alb[3];
    orc_transfer(s, orc_density(s, xs), &sig, alb);
    tau += sig * l;
  }
  return exp(-tau);
}

/* ------------------------------------------------------------------ photon cache gather */
void orc_cache_gather_bin(const orc_cache *c, int bin, const double x[3], double out[3]) {
  int n[3] = {c->res, c->res, c->res};
  double xc[3];
  for (int a = 0; a < 3; ++a) xc[a] = fmin(1.0, fmax(0.0, x[a]));
  int i0[3], i1[3];
  double f[3];
  orc_cell_corners(xc, n, i0, i1, f);
  const double *base = c->data + (size_t)bin * (size_t)c->res * c->res * c->res * 3;
  out[0] = out[1] = out[2] = 0.0;
  for (int k = 0; k < 8; ++k) {
    int ix = (k & 1) ? i1[0] : i0[0];
    int iy = (k & 2) ? i1[1] : i0[1];
    int iz = (k & 4) ? i1[2] : i0[2];
    double w = ((k & 1) ? f[0] : 1.0 - f[0]) * ((k & 2) ? f[1] : 1.0 - f[1]) *
               ((k & 4) ? f[2] : 1.0 - f[2]);
    const double *e = base + (((size_t)iz * c->res + iy) * c->res + ix) * 3;
    for (int ch = 0; ch < 3; ++ch) out[ch] += w * e[ch];
  }
}

void orc_cache_gather(const orc_cache *c, const double x[3], double g, double out[3]) {
  int nb = c->n_bins;
  if (nb == 1 || g <= c->g_bins[0]) {
    orc_cache_gather_bin(c, 0, x, out);
    return;
  }
  if (g >= c->g_bins[nb - 1]) {
    orc_cache_gather_bin(c, nb - 1, x, out);
    return;
  }
  int b = 0;
  while (b + 1 < nb - 1 && g >= c->g_bins[b + 1]) ++b;
  double w = (g - c->g_bins[b]) / (c->g_bins[b + 1] - c->g_bins[b]);
  double lo[3], hi[3];
  orc_cache_gather_bin(c, b, x, lo);
  orc_cache_gather_bin(c, b + 1, x, hi);
  for (int ch = 0; ch < 3; ++ch) out[ch] = (1.0 - w) * lo[ch] + w * hi[ch];
}

/* ------------------------------------------------------------------ metrics */
void orc_image_error(int64_t n, const double *img, const double *ref, double *rmse, double *rel_rmse,
                     double *psnr) {
  double se = 0.0, sr = 0.0, mx = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double d = img[i] - ref[i];
    se += d * d;
    sr += ref[i];
    if (ref[i] > mx) mx = ref[i];
  }
  double r = sqrt(se / (double)n);
  *rmse = r;
  *rel_rmse = r / (sr / (double)n);
  *psnr = 20.0 * log10(mx / r);
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
