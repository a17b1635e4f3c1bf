// Ray-march launch description (internal).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/pfn.h"
#include "pfn_device.h"
#include "pfn_field_dev.h"

#define PFN_MAX_LIGHTS 4

// One frame of a (batched) render.  right/up are pre-scaled by tan(fov/2)*aspect and tan(fov/2).
struct MarchJob {
  float eye[3], fwd[3], right[3], up[3];
  int width, height, spp, max_steps, stride, light_mask, slot;
  float step, t_min, g, inv_spp;
  int bin0, bin1;  // cache bins around g and the weight of bin1
  float wbin;
  uint64_t seed;
  float *out;
  int block_begin, blocks_x;
  // wavefront launch: rays of this job are [ray_begin, ray_begin + spp * tiles * 64), sample
  // major, then 64-pixel tiles in row-major tile order, then lanes inside the tile
  int64_t ray_begin;
  int tiles_x, tiles;
};

struct MarchArgs {
  const void *vol;
  BrickGrid vg;
  const uint2 *qvol;  // binary16 volumes: quad copy for two-load lookups (else null)
  BrickGrid qg;
  const float4 *tf;
  float ext_scale;
  int n_lights;
  float light_pos[PFN_MAX_LIGHTS][3], light_int[PFN_MAX_LIGHTS][3];
  const ushort4 *lightvol;
  BrickGrid lvg;
  const uint32_t *lquad;  // up to 3 lights: quad copy of the light volume (else null)
  BrickGrid lqg;
  const float4 *cache;
  int cache_res;
  const FieldDev *fields;        // per field slot
  const void *const *mlp;        // packed weights per slot
  int mlp_bytes;
  const MarchJob *jobs;
  int n_jobs, total_blocks;
  int tile_w, tile_h, block_w, block_h;  // lanes per tile row/column, tiles per block row/column
  unsigned long long *counters;          // optional: [0] march steps, [1] field/cache queries
  int persistent;                        // 0: one workgroup per block; k > 0: k workgroups per CU
  unsigned *queues;                      // 8 per-XCD block counters (persistent mode)
};

hipError_t launch_march(const MarchArgs &a, pfn_dtype vol_dtype, int direct, int ind, int prec,
                        hipStream_t st);
