// Photon tracing launch descriptions (internal).
#pragma once
#include "pfn_device.h"

struct TraceArgs {
  const void *vol;
  BrickGrid vg;
  const float4 *tf;
  float ext_scale, majorant;
  int n_lights;
  float light_pos[4][3], light_int[4][3];
  int n_bins;
  float g_bins[8];
  int max_collisions, rr_start;
  uint64_t seed, n_photons;
  float *rec_x, *rec_w, *rec_p;
  int32_t *rec_bin;
  uint8_t *rec_count;
  double *tally;
};

struct SplatArgs {
  const void *vol;
  BrickGrid vg;
  const float4 *tf;
  float ext_scale;
  int res, max_collisions;
  uint64_t n_photons;
  const float *rec_x, *rec_p;
  const int32_t *rec_bin;
  const uint8_t *rec_count;
  float4 *cache;
};

struct RecordCopyArgs {
  const uint8_t *cnt;
  uint64_t n;
  int per_block, maxrec;
  const unsigned long long *block_offsets;
  uint64_t capacity;
  const float *src_x, *src_w, *src_p;
  const int32_t *src_bin;
  float *x, *w, *p;
  int32_t *bin;
  int64_t *photon;
};
