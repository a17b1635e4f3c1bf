/*
 * FP64 oracle, photon field (test infrastructure only; see oracle.h).
 *
 *  - Field P(x, g, w) -> RGB, Eq. (2), representing the in-scattered indirect radiance of
 *    Eq. (4).
 *  - Model (Section 3.4): separate multi-resolution grid encodings for position (3-D) and
 *    direction (2-D, normalised spherical coordinates), g passed through unencoded, an MLP with
 *    ReLU between hidden layers and a linear output.  The grid encoding follows Mueller et al.,
 *    "Instant Neural Graphics Primitives with a Multiresolution Hash Encoding" (2022), Section 3:
 *    per level a grid of resolution N_l, d-linear interpolation of the features at the cell's
 *    corners, a dense table when the level's (N_l+1)^d vertices fit the table, otherwise the
 *    spatial hash XOR_i(v_i * pi_i) mod T with pi = (1, 2654435761, 805459861).
 *  - Log target encoding Eq. (6) and exponential decode Eq. (7).
 *  - Loss, Adam and the learning-rate schedule of Section 3.5.1.
 *  - Training batches of Section 3.3: uniform positions, uniform directions, g drawn from the
 *    phase pool, targets from the photon cache, a new batch every step.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle_internal.h"

/* ------------------------------------------------------------------ rounding */
/* Round to the nearest value with `mant` explicit mantissa bits and minimum normal exponent
 * emin (ties to even), i.e. IEEE binary16 (10, -14) or bfloat16 (7, -126). */
static double round_to_format(double v, int mant, int emin, double maxval) {
  if (v == 0.0 || !isfinite(v)) return v;
  double a = fabs(v);
  int e;
  frexp(a, &e); /* a = m * 2^e, m in [0.5, 1): leading bit weight 2^(e-1) */
  int lead = e - 1;
  if (lead < emin) lead = emin;
  double quantum = ldexp(1.0, lead - mant);
  double r = rint(a / quantum) * quantum; /* default rounding mode: ties to even */
  if (r > maxval) r = INFINITY;
  return v < 0.0 ? -r : r;
}

double orc_round_half(double v) { return round_to_format(v, 10, -14, 65504.0); }
double orc_round_bf16(double v) { return round_to_format(v, 7, -126, 3.3895313892515355e38); }

static inline double rnd(double v, int rounding) {
  if (rounding == 1) return orc_round_half(v);
  if (rounding == 2) return orc_round_bf16(v);
  return v;
}

/* ------------------------------------------------------------------ layout */
int orc_field_make_layout(const orc_field_desc *d, orc_field_layout *L) {
  if (d->levels < 1 || d->levels > 32 || d->feats < 1 || d->hidden_layers < 1 ||
      d->hidden_layers > 7 || d->width < 1 || d->log2_table < 1 || d->log2_table > 30)
    return -1;
  memset(L, 0, sizeof(*L));
  size_t table = (size_t)1 << d->log2_table;
  size_t off = 0;
  double r = (double)d->base_res;
  for (int l = 0; l < d->levels; ++l) {
    int res = (int)floor(r);
    size_t dense = (size_t)(res + 1) * (res + 1) * (res + 1);
    L->pos_res[l] = res;
    L->pos_dense[l] = dense <= table;
    L->pos_off[l] = off;
    off += L->pos_dense[l] ? dense : table;
    r *= d->growth;
  }
  L->pos_off[d->levels] = off;
  L->pos_params = off * (size_t)d->feats;
  off = 0;
  r = (double)d->base_res;
  for (int l = 0; l < d->levels; ++l) {
    int res = (int)floor(r);
    size_t dense = (size_t)(res + 1) * (res + 1);
    L->dir_res[l] = res;
    L->dir_dense[l] = dense <= table;
    L->dir_off[l] = off;
    off += L->dir_dense[l] ? dense : table;
    r *= d->growth;
  }
  L->dir_off[d->levels] = off;
  L->dir_params = off * (size_t)d->feats;
  L->n_in = 2 * d->levels * d->feats + 1;
  L->mlp_off = L->pos_params + L->dir_params;
  L->n_mats = d->hidden_layers + 1;
  size_t w = L->mlp_off;
  for (int m = 0; m < L->n_mats; ++m) {
    L->w_rows[m] = (m == L->n_mats - 1) ? 3 : d->width;
    L->w_cols[m] = (m == 0) ? L->n_in : d->width;
    L->w_off[m] = w;
    w += (size_t)L->w_rows[m] * L->w_cols[m];
  }
  L->n_params = w;
  return 0;
}

size_t orc_field_num_params(const orc_field_desc *d) {
  orc_field_layout L;
  if (orc_field_make_layout(d, &L)) return 0;
  return L.n_params;
}

/* ------------------------------------------------------------------ encoding */
static inline uint32_t hash3(uint32_t x, uint32_t y, uint32_t z) {
  return (x * 1u) ^ (y * 2654435761u) ^ (z * 805459861u);
}
static inline uint32_t hash2(uint32_t x, uint32_t y) { return (x * 1u) ^ (y * 2654435761u); }

/* Per corner of each level: table entry index and interpolation weight. */
typedef struct {
  size_t entry[32][8];
  double w[32][8];
} enc_pos_corners;
typedef struct {
  size_t entry[32][4];
  double w[32][4];
} enc_dir_corners;

static void pos_corners(const orc_field_desc *d, const orc_field_layout *L, const double xin[3],
                        enc_pos_corners *pc) {
  uint32_t mask = (uint32_t)(((size_t)1 << d->log2_table) - 1);
  double x[3];
  for (int a = 0; a < 3; ++a) x[a] = fmin(1.0, fmax(0.0, xin[a]));
  for (int l = 0; l < d->levels; ++l) {
    int N = L->pos_res[l];
    int c[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
      double y = x[a] * (double)N;
      double fl = floor(y);
      if (fl > (double)(N - 1)) fl = (double)(N - 1);
      c[a] = (int)fl;
      f[a] = y - fl;
    }
    for (int k = 0; k < 8; ++k) {
      uint32_t vx = (uint32_t)(c[0] + (k & 1)), vy = (uint32_t)(c[1] + ((k >> 1) & 1)),
               vz = (uint32_t)(c[2] + ((k >> 2) & 1));
      size_t idx;
      if (L->pos_dense[l])
        idx = (size_t)vx + (size_t)vy * (N + 1) + (size_t)vz * (N + 1) * (N + 1);
      else
        idx = hash3(vx, vy, vz) & mask;
      pc->entry[l][k] = L->pos_off[l] + idx;
      pc->w[l][k] = ((k & 1) ? f[0] : 1.0 - f[0]) * (((k >> 1) & 1) ? f[1] : 1.0 - f[1]) *
                    (((k >> 2) & 1) ? f[2] : 1.0 - f[2]);
    }
  }
}

/* Normalised spherical coordinates of a unit direction: (theta/pi, (phi+pi)/(2pi)). */
static void dir_coords(const double w[3], double u[2]) {
  double z = fmin(1.0, fmax(-1.0, w[2]));
  u[0] = acos(z) / M_PI;
  u[1] = (atan2(w[1], w[0]) + M_PI) / (2.0 * M_PI);
  for (int a = 0; a < 2; ++a) u[a] = fmin(1.0, fmax(0.0, u[a]));
}

static void dir_corners(const orc_field_desc *d, const orc_field_layout *L, const double w[3],
                        enc_dir_corners *dc) {
  uint32_t mask = (uint32_t)(((size_t)1 << d->log2_table) - 1);
  double u[2];
  dir_coords(w, u);
  for (int l = 0; l < d->levels; ++l) {
    int N = L->dir_res[l];
    int c[2];
    double f[2];
    for (int a = 0; a < 2; ++a) {
      double y = u[a] * (double)N;
      double fl = floor(y);
      if (fl > (double)(N - 1)) fl = (double)(N - 1);
      c[a] = (int)fl;
      f[a] = y - fl;
    }
    for (int k = 0; k < 4; ++k) {
      uint32_t vx = (uint32_t)(c[0] + (k & 1)), vy = (uint32_t)(c[1] + ((k >> 1) & 1));
      size_t idx;
      if (L->dir_dense[l])
        idx = (size_t)vx + (size_t)vy * (N + 1);
      else
        idx = hash2(vx, vy) & mask;
      dc->entry[l][k] = L->dir_off[l] + idx;
      dc->w[l][k] = ((k & 1) ? f[0] : 1.0 - f[0]) * (((k >> 1) & 1) ? f[1] : 1.0 - f[1]);
    }
  }
}

static void encode_with(const orc_field_desc *d, const orc_field_layout *L, const double *params,
                        int rounding, const enc_pos_corners *pc, const enc_dir_corners *dc, double g,
                        double *z) {
  int F = d->feats;
  const double *pos = params;
  const double *dirp = params + L->pos_params;
  for (int i = 0; i < L->n_in; ++i) z[i] = 0.0;
  for (int l = 0; l < d->levels; ++l) {
    for (int k = 0; k < 8; ++k)
      for (int f = 0; f < F; ++f)
        z[l * F + f] += pc->w[l][k] * rnd(pos[pc->entry[l][k] * F + f], rounding);
    for (int k = 0; k < 4; ++k)
      for (int f = 0; f < F; ++f)
        z[d->levels * F + l * F + f] += dc->w[l][k] * rnd(dirp[dc->entry[l][k] * F + f], rounding);
  }
  z[2 * d->levels * F] = g;
}

void orc_field_encode(const orc_field_desc *d, const double *params, int rounding, const double x[3],
                      const double w[3], double g, double *z) {
  orc_field_layout L;
  orc_field_make_layout(d, &L);
  enc_pos_corners *pc = (enc_pos_corners *)malloc(sizeof(enc_pos_corners));
  enc_dir_corners *dc = (enc_dir_corners *)malloc(sizeof(enc_dir_corners));
  pos_corners(d, &L, x, pc);
  dir_corners(d, &L, w, dc);
  encode_with(d, &L, params, rounding, pc, dc, g, z);
  free(pc);
  free(dc);
}

/* ------------------------------------------------------------------ MLP */
#define MAXW 128
typedef struct {
  double a[8][520]; /* layer inputs: a[0] = z, a[m] = ReLU(pre[m-1]) */
  double pre[8][MAXW];
} mlp_state;

static void mlp_forward(const orc_field_layout *L, const double *params, int rounding,
                        const double *z, mlp_state *st, double y[3]) {
  for (int i = 0; i < L->n_in; ++i) st->a[0][i] = z[i];
  for (int m = 0; m < L->n_mats; ++m) {
    const double *W = params + L->w_off[m];
    int R = L->w_rows[m], C = L->w_cols[m];
    for (int r = 0; r < R; ++r) {
      double acc = 0.0;
      for (int c = 0; c < C; ++c) acc += rnd(W[(size_t)r * C + c], rounding) * st->a[m][c];
      st->pre[m][r] = acc;
      if (m + 1 < L->n_mats) st->a[m + 1][r] = acc > 0.0 ? acc : 0.0;
    }
  }
  for (int c = 0; c < 3; ++c) y[c] = st->pre[L->n_mats - 1][c];
}

void orc_field_forward(const orc_field_desc *d, const double *params, int rounding, int64_t n,
                       const double *xyz, const double *dir, const double *g, double *out_lp) {
  orc_field_layout L;
  orc_field_make_layout(d, &L);
#pragma omp parallel
  {
    enc_pos_corners *pc = (enc_pos_corners *)malloc(sizeof(enc_pos_corners));
    enc_dir_corners *dc = (enc_dir_corners *)malloc(sizeof(enc_dir_corners));
    mlp_state *st = (mlp_state *)malloc(sizeof(mlp_state));
    double z[2 * 32 * 8 + 1];
#pragma omp for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
      pos_corners(d, &L, xyz + 3 * i, pc);
      dir_corners(d, &L, dir + 3 * i, dc);
      encode_with(d, &L, params, rounding, pc, dc, g[i], z);
      mlp_forward(&L, params, rounding, z, st, out_lp + 3 * i);
    }
    free(pc);
    free(dc);
    free(st);
  }
}

/* L2 loss mean over samples and the three channels; analytic gradient with respect to every
 * parameter (grid tables and weight matrices).  When the parameters are rounded before use, the
 * gradient is taken with the rounded values (the update applies to the unrounded master). */
/* loss 0: L2, sum (y - t)^2; loss 1: relative L2, sum (y - t)^2 / (y^2 + 0.01) with the
 * denominator held constant in the gradient (the relative MSE of Section 3.5.1 in the form of
 * the network library the paper trains with). */
double orc_field_loss_grad_mode(const orc_field_desc *d, const double *params, int rounding,
                                int loss_mode, int64_t n, const double *xyz, const double *dir,
                                const double *g, const double *target, double *grad) {
  orc_field_layout L;
  orc_field_make_layout(d, &L);
  memset(grad, 0, L.n_params * sizeof(double));
  int F = d->feats;
  size_t n_mlp = L.n_params - L.mlp_off;
  double loss = 0.0;
  double scale = 2.0 / (3.0 * (double)n);
#pragma omp parallel reduction(+ : loss)
  {
    enc_pos_corners *pc = (enc_pos_corners *)malloc(sizeof(enc_pos_corners));
    enc_dir_corners *dc = (enc_dir_corners *)malloc(sizeof(enc_dir_corners));
    mlp_state *st = (mlp_state *)malloc(sizeof(mlp_state));
    double *gmlp = (double *)calloc(n_mlp, sizeof(double));
    double z[2 * 32 * 8 + 1], y[3], delta[520], dprev[520];
#pragma omp for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
      pos_corners(d, &L, xyz + 3 * i, pc);
      dir_corners(d, &L, dir + 3 * i, dc);
      encode_with(d, &L, params, rounding, pc, dc, g[i], z);
      mlp_forward(&L, params, rounding, z, st, y);
      for (int c = 0; c < 3; ++c) {
        double e = y[c] - target[3 * i + c];
        double w = loss_mode == 1 ? 1.0 / (y[c] * y[c] + 0.01) : 1.0;
        loss += e * e * w;
        delta[c] = scale * e * w;
      }
      for (int m = L.n_mats - 1; m >= 0; --m) {
        const double *W = params + L.w_off[m];
        double *gW = gmlp + (L.w_off[m] - L.mlp_off);
        int R = L.w_rows[m], C = L.w_cols[m];
        for (int r = 0; r < R; ++r)
          for (int c = 0; c < C; ++c) gW[(size_t)r * C + c] += delta[r] * st->a[m][c];
        for (int c = 0; c < C; ++c) {
          double acc = 0.0;
          for (int r = 0; r < R; ++r) acc += rnd(W[(size_t)r * C + c], rounding) * delta[r];
          dprev[c] = acc;
        }
        if (m > 0)
          for (int c = 0; c < C; ++c) delta[c] = st->pre[m - 1][c] > 0.0 ? dprev[c] : 0.0;
      }
      /* dprev now holds dLoss/dz; scatter into the grid tables with the corner weights. */
      for (int l = 0; l < d->levels; ++l) {
        for (int k = 0; k < 8; ++k)
          for (int f = 0; f < F; ++f) {
            double v = pc->w[l][k] * dprev[l * F + f];
#pragma omp atomic
            grad[pc->entry[l][k] * F + f] += v;
          }
        for (int k = 0; k < 4; ++k)
          for (int f = 0; f < F; ++f) {
            double v = dc->w[l][k] * dprev[d->levels * F + l * F + f];
#pragma omp atomic
            grad[L.pos_params + dc->entry[l][k] * F + f] += v;
          }
      }
    }
#pragma omp critical
    for (size_t j = 0; j < n_mlp; ++j) grad[L.mlp_off + j] += gmlp[j];
    free(pc);
    free(dc);
    free(st);
    free(gmlp);
  }
  return loss / (3.0 * (double)n);
}

/* ------------------------------------------------------------------ target encoding */
double orc_log_encode(double v, double psi) {
  if (v > pow(10.0, -psi)) return -log10(v) / psi;
  return 1.0;
}

double orc_exp_decode(double lp, double psi) { return pow(10.0, -psi * lp); }

/* ------------------------------------------------------------------ optimiser */
void orc_adam_step(int64_t n, double *param, const double *grad, double *m, double *v, int64_t t,
                   double lr, double beta1, double beta2, double eps) {
  double bc1 = 1.0 - pow(beta1, (double)t);
  double bc2 = 1.0 - pow(beta2, (double)t);
  for (int64_t i = 0; i < n; ++i) {
    m[i] = beta1 * m[i] + (1.0 - beta1) * grad[i];
    v[i] = beta2 * v[i] + (1.0 - beta2) * grad[i] * grad[i];
    double mh = m[i] / bc1;
    double vh = v[i] / bc2;
    param[i] -= lr * mh / (sqrt(vh) + eps);
  }
}

/* Exponential decay by `decay` once at start_step and then every `interval` steps. */
double orc_lr_at(int64_t step, double lr0, double decay, int64_t start_step, int64_t interval) {
  if (step < start_step) return lr0;
  int64_t k = 1 + (step - start_step) / interval;
  return lr0 * pow(decay, (double)k);
}

/* ------------------------------------------------------------------ training batches */
/* A batch of Section 3.5.1: uniform positions and directions, and for each sample a phase value
 * and its target, Eq. (6) of the cache value over kappa.  g_mode 0 takes g from the phase pool
 * (a uniformly drawn bin, the target that bin's gather); g_mode 1 turns the same uniform draw
 * into g uniform over [g_0, g_last] and takes as target the gather interpolated linearly in g
 * between the two neighbouring bins (the same interpolation as the renderer's cache gather),
 * reporting the lower bin.  Samples first .. first + n - 1 of the batch go to rows 0 .. n - 1
 * (sample i draws from counter (step, i)). */
void orc_train_batch_range(uint64_t seed, int64_t step, int64_t first, int64_t n,
                           const orc_cache *cache, double kappa, double psi, int g_mode,
                           double *xyz, double *dir, double *g, int *bin, double *target) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    orc_rng r;
    orc_rng_init(&r, seed, ((uint64_t)step << 32) | (uint64_t)(uint32_t)(first + i),
                 ORC_STREAM_TRAIN);
    double x[3];
    for (int a = 0; a < 3; ++a) x[a] = orc_rng_next(&r);
    const double u = orc_rng_next(&r);
    double u1 = orc_rng_next(&r), u2 = orc_rng_next(&r);
    double w[3];
    orc_iso_dir(u1, u2, w);
    for (int a = 0; a < 3; ++a) {
      xyz[3 * i + a] = x[a];
      dir[3 * i + a] = w[a];
    }
    double v[3];
    int b;
    if (g_mode == 1 && cache->n_bins > 1) {
      const double g0 = cache->g_bins[0], g1 = cache->g_bins[cache->n_bins - 1];
      const double gg = g0 + u * (g1 - g0);
      b = 0;
      while (b + 2 < cache->n_bins && gg >= cache->g_bins[b + 1]) ++b;
      g[i] = gg;
      orc_cache_gather(cache, x, gg, v);
    } else {
      b = (int)floor(u * cache->n_bins);
      if (b > cache->n_bins - 1) b = cache->n_bins - 1;
      g[i] = cache->g_bins[b];
      orc_cache_gather_bin(cache, b, x, v);
    }
    if (bin) bin[i] = b;
    for (int c = 0; c < 3; ++c) target[3 * i + c] = orc_log_encode(v[c] / kappa, psi);
  }
}

void orc_train_batch_mode(uint64_t seed, int64_t step, int64_t n, const orc_cache *cache,
                          double kappa, double psi, int g_mode, double *xyz, double *dir,
                          double *g, int *bin, double *target) {
  orc_train_batch_range(seed, step, 0, n, cache, kappa, psi, g_mode, xyz, dir, g, bin, target);
}

void orc_train_batch(uint64_t seed, int64_t step, int64_t n, const orc_cache *cache, double kappa,
                     double psi, double *xyz, double *dir, double *g, int *bin, double *target) {
  orc_train_batch_mode(seed, step, n, cache, kappa, psi, 0, xyz, dir, g, bin, target);
}

double orc_field_loss_grad(const orc_field_desc *d, const double *params, int rounding, int64_t n,
                           const double *xyz, const double *dir, const double *g,
                           const double *target, double *grad) {
  return orc_field_loss_grad_mode(d, params, rounding, 0, n, xyz, dir, g, target, grad);
}
