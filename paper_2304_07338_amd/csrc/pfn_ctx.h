// Host-side context of the library (internal).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pfn.h"
#include "march.h"
#include "pfn_device.h"
#include "pfn_field_dev.h"

#define PFN_MAX_FIELDS 8
// A dispatch's grid holds fewer than 2^32 work-items per dimension (the dispatch packet's grid
// size is a 32-bit count), so launches over batches that may be larger are split into pieces of
// at most this many work-items.
#define PFN_DISPATCH_ITEMS ((int64_t)1 << 30)

struct FieldSlot {
  bool init = false;
  pfn_field_desc desc{};
  GridLevels pos{}, dir{};
  size_t pos_entries = 0, dir_entries = 0;  // table entries (2 features each)
  size_t n_params = 0, mlp_off = 0;         // floats
  size_t w_off[PFN_MAX_HIDDEN + 1] = {};    // float offset of each weight matrix
  float *master = nullptr;                  // FP32 parameters
  float *adam_m = nullptr, *adam_v = nullptr;
  float *grad = nullptr;
  uint32_t *lp_table[3] = {nullptr, nullptr, nullptr};  // packed 16-bit grid copies (f16, bf16)
  void *mlp_packed[3] = {nullptr, nullptr, nullptr};    // LDS images per precision
  bool lp_valid[3] = {false, false, false};
  void *mlp_bwd[3] = {nullptr, nullptr, nullptr};       // transposed images for training
  bool bwd_valid[3] = {false, false, false};
  int64_t adam_t = 0;
  double kappa = 1.0;
};

struct TileConfig {
  int tile_w = 8, tile_h = 8, block_w = 2, block_h = 2;
  int persistent = 0;  // 0: one workgroup per block; k: k persistent workgroups per CU
  int strategy = 0;    // render form the autotuner chose (pfn_strategy)
};

// Autotuner result for one batch shape and render form (fused with or without graph replay,
// wavefront, serial wavefront).
// Photon map (Eq. 5): records counting-sorted by (HG bin, cell of a grid^3 grid), each as
// position + red score, direction + green score, blue score (score = Phi / sigma_t).
#define PM_SCAN_DEPTH 3
struct PhotonMapState {
  float4 *ra = nullptr, *rb = nullptr;
  float *rc = nullptr;
  uint32_t *start = nullptr;   // first record of every key, n_bins * grid^3 + 1 entries
  uint32_t *counts = nullptr, *keys = nullptr;
  uint32_t *scan_tmp[PM_SCAN_DEPTH] = {};
  uint64_t n = 0, rec_cap = 0, slot_cap = 0, key_cap = 0;
  int grid = 0, n_bins = 0;
  float g_bins[8] = {};
  bool valid = false;
};
// Records to build a photon map from: trace slots (cnt, maxrec) or a dense array (cnt NULL).
struct PmSrcHost {
  const float *x, *w, *p;
  const int32_t *bin;
  const uint8_t *cnt;
  int maxrec;
  uint64_t n_slots;
};

struct TunedEntry {
  std::vector<unsigned char> key;
  TileConfig best;
  double ms = 0.0;
};

// A captured ray-march launch, replayed while its launch arguments stay the same.
struct MarchGraph {
  std::vector<unsigned char> key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

// Buffers of one round of the wavefront render (two sets, so that the march kernel of the next
// round can run while the encoding and field kernels of this one do).
struct WfRound {
  uint32_t *ent_ray = nullptr;
  int *ent_cnt = nullptr;
  int *ent_next = nullptr;
  float2 *ent_u = nullptr;
  uint32_t *ent_mask = nullptr;  // first-interaction renderer: which samples of the entry collided
  float *slot[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};  // x y z, W rgb
  void *feat = nullptr;   // position features [level][slot]
  void *dfeat = nullptr;  // direction features [level][entry]
  unsigned *count = nullptr;  // continuing rays appended by the round's march kernel
};

// Buffers of the wavefront render, kept in the context and grown on demand.
struct WfState {
  WfRound rb[2];
  uint32_t *list_ray[2] = {nullptr, nullptr};  // continuing rays, ping-pong between rounds
  int *list_j[2] = {nullptr, nullptr};
  float *list_T[2] = {nullptr, nullptr};
  float *list_cd[2] = {nullptr, nullptr};      // carried direct and indirect RGB sums
  float *list_ci[2] = {nullptr, nullptr};
  float *acc_d = nullptr, *acc_i = nullptr;    // final sums per ray sample
  unsigned *host_count = nullptr;              // pinned copies of the round counters
  int64_t *pix_begin = nullptr;
  size_t pix_cap = 0, ent_cap = 0, feat_elem = 0, acc_cap = 0;
  hipStream_t side = nullptr;                  // encoding kernels
  hipStream_t side2 = nullptr;                 // field kernels
  hipEvent_t ev_march[2] = {nullptr, nullptr}, ev_field[2] = {nullptr, nullptr}, ev_done = nullptr;
  hipEvent_t ev_enc[2] = {nullptr, nullptr};
};

#define PFN_TIMED_KERNELS 16

struct pfn_context {
  int device = 0;
  hipStream_t stream = nullptr;  // nullptr = the device's null stream
  std::string err;

  // scene
  void *vol = nullptr;
  pfn_dtype vol_dtype = PFN_F32;
  BrickGrid vol_grid{};
  size_t vol_elems = 0;
  uint2 *qvol = nullptr;     // binary16 volumes: the four (x, y) corners of every cell
  BrickGrid qvol_grid{};     // (sizes nx+1, ny+1, nz), for two-load density lookups
  size_t qvol_elems = 0;
  uint4 *cvol = nullptr;     // binary16 volumes: the eight corners of every cell, for the light
  BrickGrid cvol_grid{};     // march's one-load lookups (sizes nx+1, ny+1, nz+1); built with the
  size_t cvol_elems = 0;     // first light volume of a volume and kept while the volume stays
  bool cvol_valid = false;
  int nmax = 0;
  float4 *tf_dev = nullptr;
  float tf_host[1024] = {};
  float ext_scale = 0.0f;
  bool tf_set = false;
  float majorant = 0.0f;
  pfn_point_light lights[PFN_MAX_LIGHTS] = {};
  int n_lights = 0;

  // light-transmittance volume: 4 x f16 per texel (one channel per light)
  ushort4 *lightvol = nullptr;
  BrickGrid lv_grid{};
  size_t lv_elems = 0;
  uint32_t *lquad = nullptr;   // up to 3 lights: channels 0-2 of the four (x, y) corner texels
  BrickGrid lquad_grid{};      // of every light-volume cell (6 dwords), for four-load lookups
  size_t lquad_elems = 0;
  int lquad_lights = 0;        // lights the copy was built for (0: none)
  bool lv_valid = false;

  // photon cache: float4 (RGB, pad) per cell, [bins][res^3] x fastest
  float4 *cache = nullptr;
  int cache_bins = 0, cache_res = 0;
  float g_bins[8] = {};
  double kappa = 0.0;
  bool cache_valid = false;

  // photon records of the last trace (SoA) and their count
  // photon records of the last trace: fixed slots photon * (max_collisions - 1) + k
  float *rec_x = nullptr, *rec_w = nullptr, *rec_p = nullptr;
  int32_t *rec_bin = nullptr;
  uint8_t *rec_cnt = nullptr;   // records per photon
  uint64_t rec_cap = 0, cnt_cap = 0, rec_count = 0, rec_photons = 0;
  int rec_maxrec = 0;

  FieldSlot fields[PFN_MAX_FIELDS];
  int cur_field = 0;

  // render launch state
  MarchJob *jobs_dev = nullptr;
  size_t jobs_cap = 0;
  FieldDev *fields_dev = nullptr;
  void **mlp_ptrs_dev = nullptr;
  unsigned *queues = nullptr;     // per-XCD block queues of the persistent launch
  TileConfig tile;
  bool use_graph = false;
  hipStream_t cap_stream = nullptr;
  std::vector<MarchGraph> graphs;
  std::vector<TunedEntry> tuned;  // autotuner cache, one entry per batch shape and render form
  int strategy = PFN_STRATEGY_AUTO;  // field renders: fused kernel or wavefront rounds
  int user_strategy = PFN_STRATEGY_AUTO;  // the caller's setting: the forms the autotuner tries
  WfState wf;
  PhotonMapState pmap;
  float *pm_batch = nullptr;  // training batch with photon-map targets
  size_t pm_batch_cap = 0;

  // training activations / deltas (neuron-major, 16-bit or FP32)
  void *train_act = nullptr;
  size_t train_act_bytes = 0;

  // scratch for reductions and counters
  void *scratch = nullptr;
  size_t scratch_bytes = 0;

  // optional per-render counters (march steps, indirect queries)
  bool counting = false;
  unsigned long long *counters = nullptr;
  unsigned long long last_counts[2] = {0, 0};

  // timing: event pairs recorded around launches, collected when the totals are read
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;      // 2 events per slot
  std::vector<int> ev_kernel;           // kernel id of each pending slot
  int ev_pending = 0;
  int ev_open = 0;
  double t_ms[PFN_TIMED_KERNELS] = {};
  int64_t t_n[PFN_TIMED_KERNELS] = {};
};

enum TimedKernel {
  TK_MARCH = 0, TK_TRACE = 1, TK_TRAIN = 2, TK_PT = 3, TK_QUERY = 4, TK_ADAM = 5,
  TK_WF_MARCH = 6, TK_WF_ENCODE = 7, TK_WF_FIELD = 8, TK_WF_RESOLVE = 9, TK_FI_SAMPLE = 10,
  TK_FI_NEE = 11, TK_PM_ESTIMATE = 12, TK_WF_DIR = 13
};

// Error helpers
pfn_status pfn_fail(pfn_context *ctx, pfn_status st, const std::string &msg);
pfn_status pfn_hip(pfn_context *ctx, hipError_t e, const char *what);
#define PFN_HIP(ctx, call)                                     \
  do {                                                         \
    hipError_t e_ = (call);                                    \
    if (e_ != hipSuccess) return pfn_hip((ctx), e_, #call);    \
  } while (0)

pfn_status ensure_scratch(pfn_context *ctx, size_t bytes);
// Resolves (once per device, with that device current) the device address of the fixed scratch
// array behind pfn_image_error_noalloc.
hipError_t pfn_noalloc_init(int device);
pfn_status run_wavefront(pfn_context *ctx, const MarchArgs &m, std::vector<MarchJob> &mj,
                         int direct, int prec, int slot, const FieldDev &fd_host, bool overlap);
void wf_release(WfState &w);
int timing_begin(pfn_context *ctx);
void timing_end(pfn_context *ctx, int slot, int kernel);
int timing_begin_on(pfn_context *ctx, hipStream_t stream);
void timing_end_on(pfn_context *ctx, int slot, int kernel, hipStream_t stream);

// Kernel launchers (defined in the .hip files); all enqueue on ctx->stream.
hipError_t launch_quad_volume(pfn_context *ctx);
hipError_t launch_cube_volume(pfn_context *ctx);
hipError_t launch_light_quad(pfn_context *ctx);
hipError_t launch_brick_volume(pfn_context *ctx, const void *src, pfn_dtype dt, int nx, int ny,
                               int nz);
hipError_t launch_light_volume(pfn_context *ctx, float step);
hipError_t launch_light_unbrick(pfn_context *ctx, void *out);
hipError_t launch_field_pack(pfn_context *ctx, FieldSlot &f, int prec);
hipError_t launch_field_pack_mlp(pfn_context *ctx, FieldSlot &f, int prec);
hipError_t launch_field_pack_bwd(pfn_context *ctx, FieldSlot &f, int prec);
hipError_t launch_field_init(pfn_context *ctx, FieldSlot &f, uint64_t seed);
hipError_t launch_field_query(pfn_context *ctx, const FieldSlot &f, int prec, const float *xyz,
                              const float *dir, const float *g, int64_t n, float *lp, float *rgb);
FieldDev make_field_dev(const FieldSlot &f, int prec);
pfn_status field_refresh(pfn_context *ctx, FieldSlot &f, int prec);
void field_params_changed(FieldSlot &f);
pfn_status alloc_cache(pfn_context *ctx, int n_bins, int res);
pfn_status run_march(pfn_context *ctx, const pfn_render_job *jobs, int n_jobs, const TileConfig &tc,
                     bool first_interaction = false);
// Photon map: build (synchronises) and the Eq. (5) estimate kernel.
pfn_status pm_build(pfn_context *ctx, const PmSrcHost &src, int n_bins, const float *g_bins, int G);
hipError_t pm_launch_estimate(pfn_context *ctx, const float *xyz, const float *dir,
                              const int32_t *bin, int64_t n, float radius, int k, float *out,
                              float *r_out, int32_t *n_out, hipStream_t st);
hipError_t pm_launch_unpack(pfn_context *ctx, float *pos, float *dir, float *score, uint64_t n);
void pm_release(PhotonMapState &m);
// First-interaction renderer (one job): sampling, direct light, field pass and resolve.
pfn_status run_first_interaction(pfn_context *ctx, const MarchArgs &m, MarchJob job, int indirect,
                                 int prec, int slot, const FieldDev &fd_host);
hipError_t launch_cache_pack(pfn_context *ctx, const float *src, size_t cells);
hipError_t launch_cache_unpack(pfn_context *ctx, float *dst, size_t cells);
pfn_status count_records(pfn_context *ctx, uint64_t *out);
