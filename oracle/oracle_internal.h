/* Internal helpers of the FP64 oracle (test infrastructure only). */
#ifndef PFN_ORACLE_INTERNAL_H
#define PFN_ORACLE_INTERNAL_H
#include <math.h>
#include <stdint.h>
#include "oracle.h"

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* Philox stream: counter = (item lo, item hi, stream id, block), key = (seed lo, seed hi). */
typedef struct {
  uint32_t ctr[4];
  uint32_t key[2];
  uint32_t buf[4];
  int pos;
} orc_rng;

static inline void orc_rng_init(orc_rng *r, uint64_t seed, uint64_t item, uint32_t stream_id) {
  r->key[0] = (uint32_t)seed;
  r->key[1] = (uint32_t)(seed >> 32);
  r->ctr[0] = (uint32_t)item;
  r->ctr[1] = (uint32_t)(item >> 32);
  r->ctr[2] = stream_id;
  r->ctr[3] = 0;
  r->pos = 4;
}

static inline double orc_rng_next(orc_rng *r) {
  if (r->pos == 4) {
    orc_philox4x32_10(r->ctr, r->key, r->buf);
    r->ctr[3] += 1u;
    r->pos = 0;
  }
  return orc_u01(r->buf[r->pos++]);
}

/* Stream identifiers (one per kind of random decision). */
enum {
  ORC_STREAM_TRACE = 6,
  ORC_STREAM_TRAIN = 7,
  ORC_STREAM_RENDER = 8,
  ORC_STREAM_PT = 9,
  ORC_STREAM_FI_SAMPLE = 10, /* first-interaction renderer: free-flight walks along view rays */
  ORC_STREAM_FI_NEE = 11     /* first-interaction renderer: visibility walks toward the lights */
};

static inline double orc_dot(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static inline void orc_cross(const double a[3], const double b[3], double o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
static inline void orc_normalize(double a[3]) {
  double n = sqrt(orc_dot(a, a));
  a[0] /= n;
  a[1] /= n;
  a[2] /= n;
}

/* Distance from a point inside the unit cube to its boundary along unit direction d. */
double orc_exit_distance(const double x[3], const double d[3]);
/* Trilinear interpolation over cell centres of an n[0] x n[1] x n[2] grid with clamp-to-edge. */
void orc_cell_corners(const double x[3], const int n[3], int i0[3], int i1[3], double f[3]);
/* Isotropic direction from two uniforms: z = 1 - 2 u1, phi = 2 pi u2. */
void orc_iso_dir(double u1, double u2, double out[3]);
/* Photon emission direction from a point light (cone toward the cube); returns the fraction
 * of the full sphere of directions that the cone covers. */
double orc_emit_dir(const double p[3], double u1, double u2, double out[3]);
/* Cache gather restricted to one bin. */
void orc_cache_gather_bin(const orc_cache *c, int bin, const double x[3], double out[3]);
#endif
