// First-interaction renderer of Section 3.6 (Algorithm 2): ray generation, volume sampling by
// delta tracking, one batched field inference over the compacted interactions, direct light by
// next-event estimation with delta-tracking visibility, and composition.
//
// Rays and samples.  A view ray goes through each pixel centre; its spp samples are independent
// delta-tracking walks along that ray (the paper's several "first" interactions per ray).  The
// samples of a pixel are split into groups of 16, one matrix-core tile: ray r of the frame is
// (group, pixel) in the ray layout of the wavefront marcher (group-major, then 64-pixel tiles),
// so the wavefront kernels and the resolve serve this renderer unchanged.
//
// Kernels of a chunk of at most WF_MAX_ENTRIES rays:
//   1. fi_sample_kernel: one lane per ray.  The lane walks its samples with the global majorant
//      and keeps the collisions (position, albedo) in its own staging slots; a wave then
//      compacts the rays that have a collision into the entry list (one atomic per wave) and
//      copies their slots there.  Rays without a collision store zero sums.
//   2. fi_nee_kernel: one lane per compacted entry: for each collision, a delta-tracking
//      visibility walk toward every selected light, L_d = sum I p_g(mu) V / r^2, and the sum of
//      albedo * L_d over the entry's collisions; with the photon cache as the indirect source it
//      also sums albedo * gather(x).  It runs on a second stream beside step 3.
//   3. with the photon field: the position-encoding, direction-encoding and field kernels of the
//      wavefront marcher (weights W = albedo) store sum albedo * L_i per entry.
// After the last chunk, the resolve kernel averages (direct + indirect) over the pixel's groups
// and divides by spp (Composition, with MIS weights 1: point lights cannot be reached by phase
// sampling).
//
// Random numbers: the walk of sample s of pixel p uses Philox item p * spp + s of stream
// STREAM_FI_SAMPLE, and the visibility walks from its collision item p * spp + s of stream
// STREAM_FI_NEE (an entry keeps the mask of its group's samples that collided, so the k-th
// collision is known to be that of the k-th set bit).  Per-ray results do not depend on the
// entry a ray gets, so frames are deterministic.
#include "wavefront.h"

#define FI_GROUP 16  // samples of a pixel per ray of the layout
static_assert(FI_GROUP <= WF_SLOTS, "a sample group must fit the query slots of an entry");

#ifndef FI_GROUPED_QUERIES
#define FI_GROUPED_QUERIES (1 << 21)  // query slots from which the encoding runs per level group
#endif

struct FiArgs {
  MarchArgs m;
  MarchJob job;      // job.spp: sample groups per pixel
  float majorant;    // global majorant of sigma_t
  int spp;           // samples per pixel
  uint32_t ray0;     // first ray of the chunk
  int n_rays;
  int indirect;      // PFN_INDIRECT_*
  // staging: collisions of chunk ray i in slots wf_slot(i, k)
  float *sx, *sy, *sz, *sr, *sg, *sb;
  // compacted entries
  uint32_t *ent_ray;
  int *ent_cnt;
  int *ent_next;
  float2 *ent_u;
  uint32_t *ent_mask;  // bit s - 16 grp: sample s of the entry's group collided
  float *qx, *qy, *qz, *wr, *wg, *wb;
  unsigned *count;
  int n_entries;     // compacted entries of the chunk (NEE kernel)
  float *acc_d, *acc_i;
};

// Pixel and sample group of ray r (the wavefront ray layout with one job starting at ray 0).
__device__ __forceinline__ void fi_ray_pixel(const FiArgs &a, uint32_t r, int &grp, int &px,
                                             int &py) {
  const int64_t per_s = (int64_t)a.job.tiles * 64;
  grp = (int)((int64_t)r / per_s);
  const int rem = (int)((int64_t)r - (int64_t)grp * per_s);
  const int tile = rem >> 6, ln = rem & 63;
  px = (tile % a.job.tiles_x) * a.m.tile_w + ln % a.m.tile_w;
  py = (tile / a.job.tiles_x) * a.m.tile_h + ln / a.m.tile_w;
}

// View ray through the centre of pixel (px, py).
__device__ __forceinline__ f3 fi_ray_dir(const MarchJob &job, int px, int py) {
  const f3 fw = {job.fwd[0], job.fwd[1], job.fwd[2]};
  const f3 rt = {job.right[0], job.right[1], job.right[2]};
  const f3 up = {job.up[0], job.up[1], job.up[2]};
  const float sx = 2.0f * ((float)px + 0.5f) / (float)job.width - 1.0f;
  const float sy = 1.0f - 2.0f * ((float)py + 0.5f) / (float)job.height;
  return normalize3(fw + rt * sx + up * sy);
}

// Free-flight walk with the global majorant from o along d over (t, tmax): true, the collision
// distance and the optical properties there at the first real collision; false once the walk
// passes tmax.
template <typename VT>
__device__ __forceinline__ bool fi_delta_track(const FiArgs &a, const float4 *tf, f3 o, f3 d,
                                               float t, float tmax, Philox &rng, float &t_hit,
                                               float4 &op) {
  const VT *vol = reinterpret_cast<const VT *>(a.m.vol);
  for (;;) {
    t += -logf(rng.next()) / a.majorant;
    if (t >= tmax) return false;
    op = tf_lookup(tf, density_at(vol, a.m.vg, o + d * t));
    if (rng.next() < op.w * a.m.ext_scale / a.majorant) {
      t_hit = t;
      return true;
    }
  }
}

template <typename VT>
__global__ __launch_bounds__(WF_THREADS) void fi_sample_kernel(FiArgs a) {
  __shared__ float4 tf[256];
  for (int i = threadIdx.x; i < 256; i += blockDim.x) tf[i] = a.m.tf[i];
  __syncthreads();
  const int lane = lane_id();
  const int i = (int)(blockIdx.x * WF_THREADS + threadIdx.x);
  const bool active = i < a.n_rays;
  const uint32_t r = a.ray0 + (uint32_t)i;
  const MarchJob &job = a.job;
  int cnt = 0;
  uint32_t hit_mask = 0u;
  bool pixel_ok = false;
  float u0 = 0.0f, u1 = 0.0f;
  if (active) {
    int grp, px, py;
    fi_ray_pixel(a, r, grp, px, py);
    pixel_ok = px < job.width && py < job.height;
    float t0, t1;
    if (pixel_ok) {
      const f3 d = fi_ray_dir(job, px, py);
      dir_coords(d * -1.0f, u0, u1);
      const f3 eye = {job.eye[0], job.eye[1], job.eye[2]};
      if (clip_cube(eye, d, t0, t1) && a.majorant > 0.0f) {
        const uint64_t pix = (uint64_t)py * (uint64_t)job.width + (uint64_t)px;
        const int s0 = grp * FI_GROUP, s1 = min(a.spp, s0 + FI_GROUP);
        for (int smp = s0; smp < s1; ++smp) {
          Philox rng;
          rng.init(job.seed, pix * (uint64_t)a.spp + (uint64_t)smp, STREAM_FI_SAMPLE);
          float th;
          float4 op;
          if (fi_delta_track<VT>(a, tf, eye, d, t0, t1, rng, th, op)) {
            const f3 x = eye + d * th;
            const int64_t q = wf_slot(i, cnt);
            a.sx[q] = x.x;
            a.sy[q] = x.y;
            a.sz[q] = x.z;
            a.sr[q] = op.x;
            a.sg[q] = op.y;
            a.sb[q] = op.z;
            hit_mask |= 1u << (smp - s0);
            ++cnt;
          }
        }
      }
    }
  }
  // compaction of the rays with a collision (one atomic per wave)
  const uint64_t m = ballot(cnt > 0);
  if (m) {
    const int leader = __builtin_ctzll(m);
    unsigned base = 0;
    if (lane == leader) base = atomicAdd(a.count, (unsigned)__builtin_popcountll(m));
    base = __shfl(base, leader);
    if (cnt > 0) {
      const int t = (int)(base + (unsigned)__builtin_popcountll(m & ((1ull << lane) - 1ull)));
      a.ent_ray[t] = r;
      a.ent_cnt[t] = cnt;
      a.ent_next[t] = -1;
      a.ent_u[t] = make_float2(u0, u1);
      a.ent_mask[t] = hit_mask;
      for (int k = 0; k < cnt; ++k) {
        const int64_t q = wf_slot(i, k), o = wf_slot(t, k);
        a.qx[o] = a.sx[q];
        a.qy[o] = a.sy[q];
        a.qz[o] = a.sz[q];
        a.wr[o] = a.sr[q];
        a.wg[o] = a.sg[q];
        a.wb[o] = a.sb[q];
      }
    }
  }
  if (pixel_ok && cnt == 0) {
    float *ad = a.acc_d + (size_t)r * 3, *ai = a.acc_i + (size_t)r * 3;
    ad[0] = ad[1] = ad[2] = 0.0f;
    ai[0] = ai[1] = ai[2] = 0.0f;
  }
  if (pixel_ok && a.m.counters && cnt > 0) atomicAdd(&a.m.counters[1], (unsigned long long)cnt);
}

template <typename VT, int IND>
__global__ __launch_bounds__(WF_THREADS) void fi_nee_kernel(FiArgs a) {
  __shared__ float4 tf[256];
  for (int i = threadIdx.x; i < 256; i += blockDim.x) tf[i] = a.m.tf[i];
  __syncthreads();
  const int t = (int)(blockIdx.x * WF_THREADS + threadIdx.x);
  if (t >= a.n_entries) return;
  const MarchJob &job = a.job;
  const uint32_t r = a.ent_ray[t];
  const int cnt = a.ent_cnt[t];
  int grp, px, py;
  fi_ray_pixel(a, r, grp, px, py);
  const f3 wo = fi_ray_dir(job, px, py) * -1.0f;
  const uint64_t pix = (uint64_t)py * (uint64_t)job.width + (uint64_t)px;
  const float g = job.g;
  const float hg_c = (1.0f - g * g) * (0.25f / PFN_PI), hg_a = 1.0f + g * g, hg_b = 2.0f * g;
  f3 Sd = {0.f, 0.f, 0.f}, Si = {0.f, 0.f, 0.f};
  uint32_t mask = a.ent_mask[t];
  for (int k = 0; k < cnt; ++k) {
    const int64_t q = wf_slot(t, k);
    const f3 x = {a.qx[q], a.qy[q], a.qz[q]};
    const f3 alb = {a.wr[q], a.wg[q], a.wb[q]};
    const int smp = grp * FI_GROUP + __builtin_ctz(mask);  // the k-th set bit
    mask &= mask - 1u;
    Philox rng;
    rng.init(job.seed, pix * (uint64_t)a.spp + (uint64_t)smp, STREAM_FI_NEE);
    f3 Ld = {0.f, 0.f, 0.f};
    for (int l = 0; l < a.m.n_lights; ++l) {
      if (!((job.light_mask >> l) & 1)) continue;
      const f3 p = {a.m.light_pos[l][0], a.m.light_pos[l][1], a.m.light_pos[l][2]};
      const f3 v = x - p;
      const float ir = rsqrtf(dot(v, v));  // r > 0 unless a collision falls exactly on a light
      const float mu = dot(v, wo) * ir;
      const f3 dl = v * -ir;
      const float tmax = fminf(1.0f / ir, exit_distance(x, dl));
      float tb;
      float4 op;
      if (fi_delta_track<VT>(a, tf, x, dl, 0.0f, tmax, rng, tb, op)) continue;  // occluded
      const float rd = rsqrtf(fmaf(-hg_b, mu, hg_a));
      const float w = hg_c * (rd * rd * rd) * (ir * ir);
      Ld = Ld + f3{a.m.light_int[l][0], a.m.light_int[l][1], a.m.light_int[l][2]} * w;
    }
    Sd = Sd + mul(alb, Ld);
    if constexpr (IND == PFN_INDIRECT_CACHE) Si = Si + mul(alb, cache_gather(a.m, job, x));
  }
  float *ad = a.acc_d + (size_t)r * 3;
  ad[0] = Sd.x;
  ad[1] = Sd.y;
  ad[2] = Sd.z;
  if constexpr (IND != PFN_INDIRECT_FIELD) {
    float *ai = a.acc_i + (size_t)r * 3;
    ai[0] = Si.x;
    ai[1] = Si.y;
    ai[2] = Si.z;
  }
}

template <typename VT>
static void launch_nee(const FiArgs &a, int ind, hipStream_t st) {
  const dim3 grid((unsigned)((a.n_entries + WF_THREADS - 1) / WF_THREADS));
  if (ind == PFN_INDIRECT_FIELD)
    hipLaunchKernelGGL((fi_nee_kernel<VT, PFN_INDIRECT_FIELD>), grid, dim3(WF_THREADS), 0, st, a);
  else if (ind == PFN_INDIRECT_CACHE)
    hipLaunchKernelGGL((fi_nee_kernel<VT, PFN_INDIRECT_CACHE>), grid, dim3(WF_THREADS), 0, st, a);
  else
    hipLaunchKernelGGL((fi_nee_kernel<VT, PFN_INDIRECT_NONE>), grid, dim3(WF_THREADS), 0, st, a);
}

// One frame.  mj holds the one job (spp = samples per pixel); the job table at m.jobs is
// rewritten with the group count that the field and resolve kernels use.
pfn_status run_first_interaction(pfn_context *ctx, const MarchArgs &m, MarchJob job,
                                 int indirect, int prec, int slot, const FieldDev &fd_host) {
  WfState &w = ctx->wf;
  const int spp = job.spp;
  const int groups = (spp + FI_GROUP - 1) / FI_GROUP;
  const int64_t rays = (int64_t)groups * job.tiles * 64;
  const int64_t pixels = (int64_t)job.width * job.height;
  if (rays >= (int64_t)1 << 31)
    return pfn_fail(ctx, PFN_ERR_UNSUPPORTED, "first-interaction render: more than 2^31 rays");
  job.spp = groups;
  job.inv_spp = 1.0f / (float)spp;
  job.ray_begin = 0;
  // chunks of fewer rays for wider features, so that the feature buffers keep their size
  const int fg = indirect == PFN_INDIRECT_FIELD ? fd_host.fg : 1;
  const size_t entries = (size_t)std::min<int64_t>(rays, WF_MAX_ENTRIES / fg);
  const size_t fbytes = (prec == P_F32 ? 8 : 4) * (size_t)fg;
  PFN_HIP(ctx, wf_reserve(w, entries, (size_t)rays, fbytes));
  if (w.pix_cap < 2) {
    if (w.pix_begin) (void)hipFree(w.pix_begin);
    w.pix_begin = nullptr;
    w.pix_cap = 0;
    PFN_HIP(ctx, hipMalloc((void **)&w.pix_begin, sizeof(int64_t) * 2));
    w.pix_cap = 2;
  }
  const int64_t pix_begin[2] = {0, pixels};
  PFN_HIP(ctx, hipMemcpyAsync(const_cast<MarchJob *>(m.jobs), &job, sizeof(MarchJob),
                              hipMemcpyHostToDevice, ctx->stream));
  PFN_HIP(ctx, hipMemcpyAsync(w.pix_begin, pix_begin, sizeof(pix_begin), hipMemcpyHostToDevice,
                              ctx->stream));
  PFN_HIP(ctx, hipStreamSynchronize(ctx->stream));  // the host copies above go out of scope
  std::vector<std::pair<int, int>> lgroups;
  int fb_max = 1;
  if (indirect == PFN_INDIRECT_FIELD) {
    lgroups = wf_level_groups(ctx, slot, fd_host, fbytes);
    fb_max = wf_field_blocks(prec, m.mlp_bytes, fg);
  }
  hipStream_t sa = ctx->stream, sb = w.side;
  WfRound &b = w.rb[0], &st = w.rb[1];

  const int tslot = timing_begin(ctx);
  for (int64_t ray0 = 0; ray0 < rays; ray0 += (int64_t)entries) {
    FiArgs a{};
    a.m = m;
    a.job = job;
    a.majorant = ctx->majorant;
    a.spp = spp;
    a.ray0 = (uint32_t)ray0;
    a.n_rays = (int)std::min<int64_t>((int64_t)entries, rays - ray0);
    a.indirect = indirect;
    a.sx = st.slot[0];
    a.sy = st.slot[1];
    a.sz = st.slot[2];
    a.sr = st.slot[3];
    a.sg = st.slot[4];
    a.sb = st.slot[5];
    a.ent_ray = b.ent_ray;
    a.ent_cnt = b.ent_cnt;
    a.ent_next = b.ent_next;
    a.ent_mask = b.ent_mask;
    a.ent_u = b.ent_u;
    a.qx = b.slot[0];
    a.qy = b.slot[1];
    a.qz = b.slot[2];
    a.wr = b.slot[3];
    a.wg = b.slot[4];
    a.wb = b.slot[5];
    a.count = b.count;
    a.acc_d = w.acc_d;
    a.acc_i = w.acc_i;
    PFN_HIP(ctx, hipMemsetAsync(b.count, 0, 4, sa));
    {
      const int ts = timing_begin_on(ctx, sa);
      const dim3 grid((unsigned)((a.n_rays + WF_THREADS - 1) / WF_THREADS));
      if (ctx->vol_dtype == PFN_F16)
        hipLaunchKernelGGL(fi_sample_kernel<__half>, grid, dim3(WF_THREADS), 0, sa, a);
      else
        hipLaunchKernelGGL(fi_sample_kernel<float>, grid, dim3(WF_THREADS), 0, sa, a);
      timing_end_on(ctx, ts, TK_FI_SAMPLE, sa);
    }
    PFN_HIP(ctx, hipGetLastError());
    PFN_HIP(ctx, hipMemcpyAsync(w.host_count, b.count, 4, hipMemcpyDeviceToHost, sa));
    PFN_HIP(ctx, hipStreamSynchronize(sa));
    a.n_entries = (int)w.host_count[0];
    if (a.n_entries == 0) continue;

    // direct light (and the cache gather) on the side stream, the field pass on this one
    PFN_HIP(ctx, hipEventRecord(w.ev_march[0], sa));
    PFN_HIP(ctx, hipStreamWaitEvent(sb, w.ev_march[0], 0));
    {
      const int ts = timing_begin_on(ctx, sb);
      if (ctx->vol_dtype == PFN_F16) launch_nee<__half>(a, indirect, sb);
      else launch_nee<float>(a, indirect, sb);
      timing_end_on(ctx, ts, TK_FI_NEE, sb);
    }
    PFN_HIP(ctx, hipGetLastError());
    if (indirect == PFN_INDIRECT_FIELD) {
      WfEncArgs e{};
      e.F = m.fields + slot;
      e.ent_cnt = b.ent_cnt;
      e.qx = b.slot[0];
      e.qy = b.slot[1];
      e.qz = b.slot[2];
      e.feat = b.feat;
      e.n_slots = wf_slots(a.n_entries);
      e.n_entries = a.n_entries;
      e.kshift = 0;  // entries hold min(spp, 16) collisions at most
      while ((1 << e.kshift) < std::min(spp, FI_GROUP)) ++e.kshift;
      WfDirArgs dg{};
      dg.F = m.fields + slot;
      dg.ent_cnt = b.ent_cnt;
      dg.ent_u = b.ent_u;
      dg.dfeat = b.dfeat;
      dg.n_entries = a.n_entries;
      WfFieldArgs f{};
      f.F = m.fields + slot;
      f.mlp = ctx->fields[slot].mlp_packed[prec];
      f.mlp_bytes = m.mlp_bytes;
      f.jobs = m.jobs;
      f.n_jobs = 1;
      f.ent_ray = b.ent_ray;
      f.ent_cnt = b.ent_cnt;
      f.ent_next = b.ent_next;
      f.wr = b.slot[3];
      f.wg = b.slot[4];
      f.wb = b.slot[5];
      f.feat = b.feat;
      f.dfeat = b.dfeat;
      f.acc_i = w.acc_i;
      f.n_slots = e.n_slots;
      f.n_entries = a.n_entries;
      f.fg = fg;
      f.n_cont = 0;
      f.in_ci = nullptr;
      f.out_ci = nullptr;
      const int fb = std::max(1, std::min((a.n_entries + 63) / 64, fb_max));
      // first interactions of neighbouring rays lie at unrelated depths, so a query's levels
      // gain nothing from sharing a thread: one thread per (level, query).  A small pass
      // encodes every level in one launch; from FI_GROUPED_QUERIES query slots on, the level
      // groups keep each fine table resident in L2
      const bool grouped = ((int64_t)a.n_entries << e.kshift) >= FI_GROUPED_QUERIES;
      const std::vector<std::pair<int, int>> one = {{0, fd_host.levels}};
      PFN_HIP(ctx, wf_launch_field_pass(ctx, sa, prec, e, dg, grouped ? lgroups : one, f, fb, true));
      PFN_HIP(ctx, hipGetLastError());
    }
    // the next chunk rewrites the entries: wait for the direct-light kernel
    PFN_HIP(ctx, hipEventRecord(w.ev_done, sb));
    PFN_HIP(ctx, hipStreamWaitEvent(sa, w.ev_done, 0));
  }
  WfResolveArgs ra{};
  ra.jobs = m.jobs;
  ra.n_jobs = 1;
  ra.pix_begin = w.pix_begin;
  ra.acc_d = w.acc_d;
  ra.acc_i = w.acc_i;
  ra.tile_w = m.tile_w;
  ra.tile_h = m.tile_h;
  wf_launch_resolve(ctx, sa, ra, pixels);
  PFN_HIP(ctx, hipGetLastError());
  timing_end(ctx, tslot, TK_MARCH);
  return PFN_OK;
}
