// Ray-march launch description (internal).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/pfn.h"
#include "pfn_device.h"
#include "pfn_field_dev.h"

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
};

struct MarchArgs {
  const void *vol;
  BrickGrid vg;
  const float4 *tf;
  float ext_scale;
  int n_lights;
  float light_pos[4][3], light_int[4][3];
  const ushort4 *lightvol;
  BrickGrid lvg;
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
