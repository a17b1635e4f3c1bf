// Shared pieces of the wavefront renderers (internal): the query-slot layout, the arguments of
// the position-encoding, direction-encoding, field and resolve kernels, and the host helpers
// that size their buffers and launch them.  The ray marcher's wavefront form and the
// first-interaction renderer both feed these kernels.
#pragma once
#include <utility>
#include <vector>

#include "march.h"
#include "march_dev.h"
#include "pfn_ctx.h"

#define WF_THREADS 256
#ifndef WF_SLOTS_LOG2
#define WF_SLOTS_LOG2 5
#endif
#define WF_SLOTS (1 << WF_SLOTS_LOG2)  // queries per ray per round
#define WF_MAX_ENTRIES (1 << 21)     // rays per round
#define WF_FINE_RES 1024             // hashed levels from this resolution on are encoded apart
#ifndef WF_GROUP_BYTES
#define WF_GROUP_BYTES (64u << 20)   // table bytes the coarse levels of one encoding launch span
#endif

// Query slot k of round entry t.  Slots are tiled as [t / 64][k][t % 64]: the 64 rays of a wave
// write slot k of 64 consecutive entries, and 16 neighbouring rays' slot k are 64 contiguous
// bytes for the field kernel.
__host__ __device__ __forceinline__ int64_t wf_slot(int64_t t, int k) {
  return ((t >> 6) << (6 + WF_SLOTS_LOG2)) | ((int64_t)k << 6) | (t & 63);
}
// Slots spanned by the first n entries.
__host__ __device__ __forceinline__ int64_t wf_slots(int64_t n) {
  return ((n + 63) >> 6) << (6 + WF_SLOTS_LOG2);
}

struct WfEncArgs {
  const FieldDev *F;
  const int *ent_cnt;
  const float *qx, *qy, *qz;
  void *feat;           // [level][slot]: fg uint32 (pairs of 16-bit features) or fg float2
  int64_t n_slots;
  int n_entries;
  int kshift;           // entries hold at most 2^kshift queries (WF_SLOTS_LOG2: any count)
  int l0, l1;
  int per_level;        // 0: a thread encodes levels l0..l1-1 of its query; > 0: a thread
                        // encodes one level, per_level threads per level, level-major
  int xcd_levels;       // 2 or 4: levels l0 .. l0 + xcd_levels - 1, each on its own 8 /
                        // xcd_levels XCDs, so that each XCD's L2 holds one level's table
  int paired;           // 1: all levels 0 .. l1-1 (8 <= l1 <= 16) in one launch; XCD x encodes
                        // level x and, if it is 8 or more, level l1 - 1 - x
};

struct WfDirArgs {
  const FieldDev *F;
  const int *ent_cnt;
  const float2 *ent_u;
  void *dfeat;          // [level][entry]
  int n_entries;
};

struct WfFieldArgs {
  const FieldDev *F;
  const void *mlp;
  int mlp_bytes;
  const MarchJob *jobs;
  int n_jobs;
  const uint32_t *ent_ray;
  const int *ent_cnt;
  const int *ent_next;
  const float *wr, *wg, *wb;
  const void *feat, *dfeat;
  const float *in_ci;   // carried indirect sums of the continued entries [0, n_cont)
  float *out_ci;
  float *acc_i;
  int64_t n_slots;
  int n_entries, n_cont;
  int fg;               // feature groups of the field (1 or 4), host-side dispatch
};

struct WfResolveArgs {
  const MarchJob *jobs;
  int n_jobs;
  const int64_t *pix_begin;  // per job, plus the total at [n_jobs]
  const float *acc_d, *acc_i;
  int tile_w, tile_h;
};

// Job of ray r: the last job whose first ray is <= r.
__device__ __forceinline__ int find_job_ray(const MarchJob *jobs, int n_jobs, int64_t r) {
  int lo = 0, hi = n_jobs - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].ray_begin <= r) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Buffers for `entries` rays per round, `rays` ray samples per frame and feature elements of
// `feat_bytes` bytes; kept between frames and grown on demand.
hipError_t wf_reserve(WfState &w, size_t entries, size_t rays, size_t feat_bytes);
// Level groups of the position encoding of field slot `slot`: the coarse levels together (up to
// WF_GROUP_BYTES of tables), each fine hashed level alone.  The Algorithm 2 renderer launches
// these groups; the ray marcher pairs 8 to 16 levels over the XCDs in one launch and uses the
// groups (consecutive fine levels merged, each on its own XCDs) only for other level counts.
std::vector<std::pair<int, int>> wf_level_groups(const pfn_context *ctx, int slot,
                                                 const FieldDev &fd_host, size_t feat_bytes);
// Field-kernel workgroups that are resident on the device at once.
int wf_field_blocks(int prec, int mlp_bytes, int fg = 1);
// The encoding launches (one per level group), the direction encoding and the field kernel of
// one round, on stream st.
// split_levels: each group launch runs one thread per (level, query) instead of one per query.
// field_st: when set, the direction encoding and the field kernel run on that stream instead
// (which the caller has made wait for the march kernel), the field kernel after enc_done
// (recorded on st once the position encodings are done).
hipError_t wf_launch_field_pass(pfn_context *ctx, hipStream_t st, int prec, const WfEncArgs &e,
                                const WfDirArgs &dg,
                                const std::vector<std::pair<int, int>> &groups,
                                const WfFieldArgs &f, int field_blocks, bool split_levels = false,
                                hipStream_t field_st = nullptr, hipEvent_t enc_done = nullptr);
// Pixel averages over the ray samples of every job.
void wf_launch_resolve(pfn_context *ctx, hipStream_t st, const WfResolveArgs &ra, int64_t pixels);
