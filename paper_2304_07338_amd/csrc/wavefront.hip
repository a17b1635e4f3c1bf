// Wavefront form of the photon-field ray marcher (Section 3.6 with Eq. (3): the field supplies
// L_i at the samples of a ray marcher).  The fused kernel keeps a ray and its field queries in
// one wave; here a frame runs in rounds of small kernels so that each piece runs at its own
// best occupancy and the fine hash levels of the position encoding stay resident in L2:
//
//   1. wf_march_kernel: one lane per ray (a pixel sample).  The lane marches groups of `stride`
//      steps exactly as the fused kernel does (transfer function, transmittance, direct light,
//      compositing) and, for every group with a non-zero weight W = sum T*alpha*albedo, stores
//      the query (position of the group's first step, W) in the ray's next slot.  After
//      WF_SLOTS queries the ray stops and is appended to the list of rays continued next round.
//   2. wf_encode_kernel: the position encoding of every stored query, written level-major as
//      the 16-bit (or FP32) features the matrix cores consume.  One launch covers all levels:
//      XCD x encodes level x and level L-1-x, a coarse level whose neighbouring queries share
//      cells with a fine one whose queries each touch their own cache lines, so that the XCDs
//      carry similar loads and each XCD's L2 holds at most two 2 MB tables.
//      wf_dir_kernel encodes the view direction once per ray of the round.
//   3. wf_field_kernel: a wave takes 16 rays of the round: the MLP of their queries on the
//      matrix cores, one 16-query tile per query index, the Eq. (7) decode, and each ray's sum of
//      W * L_i over its queries in a fixed order.  The input layer's direction and g products
//      are the same for all tiles of the 16 rays and are computed once.
//   4. after the last round, wf_resolve_kernel averages each pixel's samples.
//
// A ray carries its direct sum and its indirect sum in the list from round to round and
// stores them once, when it ends; no kernel reads and rewrites a pixel.  Every ray's arithmetic
// is the fused kernel's; only the order in which the FP32 terms are added differs.  Results do
// not depend on the lane or list position a ray gets, so a frame is deterministic and a batch
// renders exactly as its jobs rendered alone.
#include "wavefront.h"

#ifndef WF_XCD_LEVELS
#define WF_XCD_LEVELS 4  // without pairing: fine levels per encoding launch, each on
                         // 8 / WF_XCD_LEVELS XCDs
#endif

struct WfList {
  uint32_t *ray;
  int *j;
  float *T;
  float *cd;
  float *ci;
};

struct WfArgs {
  MarchArgs m;
  WfList in, out;     // in: entries [0, n_cont); out: appended through out_count
  int n_cont, n_fresh;
  int64_t fresh_begin;
  unsigned *out_count;
  // per entry of this round
  uint32_t *ent_ray;
  int *ent_cnt;
  int *ent_next;      // the ray's index in the out list; -1: the ray ended; -2: no pixel
  float2 *ent_u;
  // per query slot (wf_slot(entry, k))
  float *qx, *qy, *qz, *wr, *wg, *wb;
  float *acc_d, *acc_i;  // per ray sample: final direct and indirect RGB sums
};

// One ray of the round (see wf_march_kernel); `job` is uniform across the calling lanes.
template <typename VT, int DIRECT>
__device__ __forceinline__ void march_entry(const WfArgs &a, const float4 *tf, const MarchJob &job,
                                            int t, bool active, uint32_t r, int j,
                                            float T, f3 Cd) {
  const int lane = lane_id();
  int px = 0, py = 0, s = 0;
  {
    const int64_t rr = (int64_t)r - job.ray_begin;
    const int64_t per_s = (int64_t)job.tiles * 64;
    s = (int)(rr / per_s);
    const int rem = (int)(rr - (int64_t)s * per_s);
    const int tile = rem >> 6, ln = rem & 63;
    px = (tile % job.tiles_x) * a.m.tile_w + ln % a.m.tile_w;
    py = (tile / job.tiles_x) * a.m.tile_h + ln / a.m.tile_w;
  }
  const bool pixel_ok = active && px < job.width && py < job.height;

  const f3 eye = {job.eye[0], job.eye[1], job.eye[2]};
  f3 d = {0.f, 0.f, 1.f}, wo = {0.f, 0.f, -1.f};
  float t0 = 0.f, span = 0.f, xi = 0.5f, u0 = 0.f, u1 = 0.f;
  int n = 0;
  bool live = false;
  if (pixel_ok) {
    float jx = 0.5f, jy = 0.5f;
    if (job.spp > 1) {
      Philox rng;
      rng.init(job.seed, ((uint64_t)py * job.width + px) * (uint64_t)job.spp + (uint64_t)s,
               STREAM_RENDER);
      jx = rng.next();
      jy = rng.next();
      xi = rng.next();
    }
    const f3 fw = {job.fwd[0], job.fwd[1], job.fwd[2]};
    const f3 rt = {job.right[0], job.right[1], job.right[2]};
    const f3 up = {job.up[0], job.up[1], job.up[2]};
    float sx = 2.0f * ((float)px + jx) / (float)job.width - 1.0f;
    float sy = 1.0f - 2.0f * ((float)py + jy) / (float)job.height;
    d = normalize3(fw + rt * sx + up * sy);
    wo = d * -1.0f;
    float t1;
    if (clip_cube(eye, d, t0, t1)) {
      span = t1 - t0;
      float ns = ceilf(span / job.step);
      n = ns > (float)job.max_steps ? job.max_steps : (int)ns;
      dir_coords(wo, u0, u1);
      live = n > j;
    }
  }

  int cnt = 0;
  bool finished = !live;
  unsigned n_steps = 0;
  while (!finished && cnt < WF_SLOTS) {
    f3 W = {0.f, 0.f, 0.f};
    f3 xq = {0.f, 0.f, 0.f};
    for (int k = 0; k < job.stride; ++k) {
      float l = fminf(job.step, span - (float)j * job.step);
      if (!(l > 0.0f)) {
        finished = true;
        break;
      }
      float tt = t0 + (float)j * job.step + xi * l;
      f3 x = eye + d * tt;
      float rho = density_march(reinterpret_cast<const VT *>(a.m.vol), a.m.vg, a.m.qvol, a.m.qg, x);
      float4 o = tf_lookup(tf, rho);
      float sig = o.w * a.m.ext_scale;
      float alpha = -expm1f(-sig * l);
      float att = 1.0f - alpha;
      f3 alb = {o.x, o.y, o.z};
      f3 Ld = direct_light<VT, DIRECT>(a.m, job, tf, x, wo);
      f3 wgt = alb * (T * alpha);
      ++n_steps;
      if (k == 0) xq = x;
      Cd = Cd + mul(wgt, Ld);
      W = W + wgt;
      T *= att;
      ++j;
      if (j >= n || T < job.t_min) {
        finished = true;
        break;
      }
    }
    if (W.x != 0.f || W.y != 0.f || W.z != 0.f) {
      const int64_t q = wf_slot(t, cnt);
      a.qx[q] = xq.x;
      a.qy[q] = xq.y;
      a.qz[q] = xq.z;
      a.wr[q] = W.x;
      a.wg[q] = W.y;
      a.wb[q] = W.z;
      ++cnt;
    }
  }
  // rays that filled their slots continue next round (one atomic per wave)
  const bool cont = pixel_ok && !finished;
  const uint64_t m = __builtin_amdgcn_ballot_w64(cont);
  int next = -1;
  if (m) {
    const int leader = __builtin_ctzll(m);
    unsigned base = 0;
    if (lane == leader) base = atomicAdd(a.out_count, (unsigned)__builtin_popcountll(m));
    base = __shfl(base, leader);
    if (cont) {
      next = (int)(base + (unsigned)__builtin_popcountll(m & ((1ull << lane) - 1ull)));
      a.out.ray[next] = r;
      a.out.j[next] = j;
      a.out.T[next] = T;
      a.out.cd[3 * (size_t)next] = Cd.x;
      a.out.cd[3 * (size_t)next + 1] = Cd.y;
      a.out.cd[3 * (size_t)next + 2] = Cd.z;
    }
  }
  if (active) {
    a.ent_cnt[t] = pixel_ok ? cnt : 0;
    a.ent_ray[t] = r;
    a.ent_next[t] = pixel_ok ? next : -2;
    a.ent_u[t] = make_float2(u0, u1);
  }
  if (pixel_ok && !cont) {
    float *ad = a.acc_d + (size_t)r * 3;
    ad[0] = Cd.x;
    ad[1] = Cd.y;
    ad[2] = Cd.z;
  }
  if (pixel_ok && a.m.counters) {
    atomicAdd(&a.m.counters[0], (unsigned long long)n_steps);
    atomicAdd(&a.m.counters[1], (unsigned long long)cnt);
  }
}

template <typename VT, int DIRECT>
__global__ __launch_bounds__(WF_THREADS) void wf_march_kernel(WfArgs a) {
  __shared__ float4 tf[256];
  for (int i = threadIdx.x; i < 256; i += blockDim.x) tf[i] = a.m.tf[i];
  __syncthreads();
  const int n_in = a.n_cont + a.n_fresh;
  const int needed = (n_in + WF_THREADS - 1) / WF_THREADS;
  // XCD-aware order: XCD x (blockIdx % 8) takes a contiguous run of entries
  const int per = (int)(gridDim.x >> 3);
  const int b = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (b >= needed) return;
  const int t = b * WF_THREADS + (int)threadIdx.x;
  const bool active = t < n_in;
  const bool fresh = t >= a.n_cont;
  uint32_t r = 0;
  int j = 0;
  float T = 1.0f;
  f3 Cd = {0.f, 0.f, 0.f};
  if (active) {
    if (!fresh) {
      r = a.in.ray[t];
      j = a.in.j[t];
      T = a.in.T[t];
      Cd = {a.in.cd[3 * (size_t)t], a.in.cd[3 * (size_t)t + 1], a.in.cd[3 * (size_t)t + 2]};
    } else {
      r = (uint32_t)(a.fresh_begin + (t - a.n_cont));
    }
  }
  // waterfall over the jobs present in the wave, so that each pass reads its job descriptor
  // into scalar registers
  const int ji = find_job_ray(a.m.jobs, a.m.n_jobs, (int64_t)r);
  for (bool pending = true; pending;) {
    const int jc = __builtin_amdgcn_readfirstlane(ji);
    if (ji == jc) {
      march_entry<VT, DIRECT>(a, tf, a.m.jobs[jc], t, active, r, j, T, Cd);
      pending = false;
    }
  }
}

template <int P>
__device__ __forceinline__ void store_feat(void *feat, int64_t i, float2 v) {
  if constexpr (P == P_F32) {
    reinterpret_cast<float2 *>(feat)[i] = v;
  } else if constexpr (P == P_F16) {
    __half2 h = __floats2half2_rn(v.x, v.y);
    reinterpret_cast<uint32_t *>(feat)[i] = *reinterpret_cast<uint32_t *>(&h);
  } else {
    __bf16 lo = (__bf16)v.x, hi = (__bf16)v.y;
    uint32_t w = (uint32_t)__builtin_bit_cast(unsigned short, lo) |
                 ((uint32_t)__builtin_bit_cast(unsigned short, hi) << 16);
    reinterpret_cast<uint32_t *>(feat)[i] = w;
  }
}

template <int P>
__device__ __forceinline__ uint32_t pack_pair(float a, float b) {
  if constexpr (P == P_F16) {
    __half2 h = __floats2half2_rn(a, b);
    return *reinterpret_cast<uint32_t *>(&h);
  } else {
    __bf16 lo = (__bf16)a, hi = (__bf16)b;
    return (uint32_t)__builtin_bit_cast(unsigned short, lo) |
           ((uint32_t)__builtin_bit_cast(unsigned short, hi) << 16);
  }
}

// 8 features of one level: 16 bytes (16-bit) or 32 bytes (FP32) at element i.
template <int P>
__device__ __forceinline__ void store_feat8(void *feat, int64_t i, const float v[8]) {
  if constexpr (P == P_F32) {
    float4 *d = reinterpret_cast<float4 *>(feat) + 2 * i;
    d[0] = make_float4(v[0], v[1], v[2], v[3]);
    d[1] = make_float4(v[4], v[5], v[6], v[7]);
  } else {
    uint4 w;
    w.x = pack_pair<P>(v[0], v[1]);
    w.y = pack_pair<P>(v[2], v[3]);
    w.z = pack_pair<P>(v[4], v[5]);
    w.w = pack_pair<P>(v[6], v[7]);
    reinterpret_cast<uint4 *>(feat)[i] = w;
  }
}

template <int P>
__device__ __forceinline__ float2 load_feat2(const void *feat, int64_t i) {
  if constexpr (P == P_F32) return reinterpret_cast<const float2 *>(feat)[i];
  else return load_feat<P>(reinterpret_cast<const uint32_t *>(feat) + i, 0u);
}

template <int P, int FG>
__global__ __launch_bounds__(WF_THREADS) void wf_encode_kernel(WfEncArgs e) {
  // thread g: query c of entry t, over the first 2^kshift query indices of every entry (and,
  // with per_level, one level of it)
  int64_t g = (int64_t)blockIdx.x * WF_THREADS + threadIdx.x;
  int l0 = e.l0, l1 = e.l1;
  if (e.paired) {
    // workgroups go to the XCDs round-robin: blockIdx % 8 is the XCD, which encodes level
    // l0 = x and, when it is not another XCD's own level, level l1 = L - 1 - x
    const int xcd = (int)(blockIdx.x & 7);
    g = (int64_t)(blockIdx.x >> 3) * WF_THREADS + threadIdx.x;
    l0 = xcd;
    l1 = e.l1 - 1 - xcd;
  } else if (e.xcd_levels) {
    // workgroups go to the XCDs round-robin: blockIdx % 8 is the XCD; level l0 + j runs on the
    // per = 8 / xcd_levels XCDs j * per .. j * per + per - 1
    const int xcd = (int)(blockIdx.x & 7), per = 8 / e.xcd_levels;
    l0 += xcd / per;
    l1 = l0 + 1;
    g = ((int64_t)(blockIdx.x >> 3) * per + (xcd % per)) * WF_THREADS + threadIdx.x;
  } else if (e.per_level) {
    const int dl = (int)(g / e.per_level);
    g -= (int64_t)dl * e.per_level;
    l0 += dl;
    l1 = l0 + 1;
    if (l0 >= e.l1) return;
  }
  const int64_t t = ((g >> (6 + e.kshift)) << 6) | (g & 63);
  const int c = (int)((g >> 6) & ((1 << e.kshift) - 1));
  if (t >= e.n_entries || c >= e.ent_cnt[t]) return;
  const int64_t s = wf_slot(t, c);
  const FieldDev &F = *e.F;
  const f3 x = clamp01(f3{e.qx[s], e.qy[s], e.qz[s]});
  if constexpr (FG != 1) {
    // 8 features per level: one 16- (or 32-) byte read per corner and one store per level
    float v[8];
    if (e.paired) {
      encode_pos_level8<P>(F, l0, x, v);
      store_feat8<P>(e.feat, (int64_t)l0 * e.n_slots + s, v);
      if (l1 >= 8) {
        encode_pos_level8<P>(F, l1, x, v);
        store_feat8<P>(e.feat, (int64_t)l1 * e.n_slots + s, v);
      }
      return;
    }
    for (int lv = l0; lv < l1; ++lv) {
      encode_pos_level8<P>(F, lv, x, v);
      store_feat8<P>(e.feat, (int64_t)lv * e.n_slots + s, v);
    }
    return;
  }
  if (e.paired) {
    // both levels' corner reads are issued before either store
    const bool two = l1 >= 8;
    const float2 va = encode_pos_level<P>(F, l0, x);
    const float2 vb = encode_pos_level<P>(F, two ? l1 : l0, x);
    store_feat<P>(e.feat, (int64_t)l0 * e.n_slots + s, va);
    if (two) store_feat<P>(e.feat, (int64_t)l1 * e.n_slots + s, vb);
    return;
  }
  for (int lv = l0; lv < l1; ++lv)
    store_feat<P>(e.feat, (int64_t)lv * e.n_slots + s, encode_pos_level<P>(F, lv, x));
}

template <int P, int FG>
__global__ __launch_bounds__(WF_THREADS) void wf_dir_kernel(WfDirArgs e) {
  const int t = (int)(blockIdx.x * WF_THREADS + threadIdx.x);
  if (t >= e.n_entries) return;
  if (e.ent_cnt[t] == 0) return;
  const FieldDev &F = *e.F;
  const float2 u = e.ent_u[t];
  if constexpr (FG != 1) {
    float v[8];
    for (int lv = 0; lv < F.levels; ++lv) {
      encode_dir_level8<P>(F, lv, u.x, u.y, v);
      store_feat8<P>(e.dfeat, (int64_t)lv * e.n_entries + t, v);
    }
    return;
  }
  for (int lv = 0; lv < F.levels; ++lv)
    store_feat<P>(e.dfeat, (int64_t)lv * e.n_entries + t,
                  encode_dir_level<P>(F, lv, u.x, u.y));
}

// Field kernel: a wave takes 16 neighbouring rays of the round (entries t0..t0+15, one per
// matrix-core column) and runs one tile per query index k < WF_SLOTS: column c of tile k is
// query k of ray t0+c.  Lane group q holds levels 4q..4q+3 of its column's features; the direction
// features of a column's ray are loaded once for all tiles.  Each column accumulates W * L_i of
// its ray over k in order, in the lanes of group 0.
// The 16-bit weights take 30 KB of LDS per workgroup, so 5 waves per SIMD are resident; the
// register budget is held to that occupancy.
template <int P>
__global__ __launch_bounds__(WF_THREADS) __attribute__((amdgpu_waves_per_eu(5, 8)))
void wf_field_kernel(WfFieldArgs a) {
  extern __shared__ __align__(16) unsigned char lds_w[];
  stage_weights(lds_w, a.mlp, a.mlp_bytes);
  __syncthreads();
  const FieldDev &F = *a.F;
  const int lane = lane_id(), q = lane >> 4, col = lane & 15;
  const int waves = (int)gridDim.x * (WF_THREADS / 64);
  const int w0 = __builtin_amdgcn_readfirstlane((int)blockIdx.x * (WF_THREADS / 64) +
                                                (int)(threadIdx.x >> 6));
  const int n_tiles = (a.n_entries + 15) >> 4;
  for (int rt = w0; rt < n_tiles; rt += waves) {
    const int t = rt * 16 + col;
    const bool tv = t < a.n_entries;
    const int cnt = tv ? a.ent_cnt[t] : 0;
    const int next = tv ? a.ent_next[t] : -2;
    int kmax = cnt;
#pragma unroll
    for (int o = 8; o >= 1; o >>= 1) kmax = max(kmax, __shfl_xor(kmax, o));
    kmax = __builtin_amdgcn_readfirstlane(kmax);
    uint32_t r = 0;
    f3 ci = {0.f, 0.f, 0.f};
    if (next != -2) {
      r = a.ent_ray[t];
      if (t < a.n_cont)
        ci = {a.in_ci[3 * (size_t)t], a.in_ci[3 * (size_t)t + 1], a.in_ci[3 * (size_t)t + 2]};
    }
    float gin = 0.0f;
    if (cnt > 0 && q == 0) gin = a.jobs[find_job_ray(a.jobs, a.n_jobs, (int64_t)r)].g;
    f3 S = {0.f, 0.f, 0.f};
    if constexpr (P == P_F32) {
      float dir[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) dir[k] = 0.0f;
      if (cnt > 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int lv = 4 * q + k;
          if (lv < F.levels) {
            const float2 fd = load_feat2<P>(a.dfeat, (int64_t)lv * a.n_entries + t);
            dir[2 * k] = fd.x;
            dir[2 * k + 1] = fd.y;
          }
        }
      }
      for (int k = 0; k < kmax; ++k) {
        int wofs = 0;  // opaque offset: keeps the LDS weight reads inside the loop
        asm volatile("" : "+s"(wofs));
        const bool valid = k < cnt;
        const int64_t sl = wf_slot(t, k);
        float pos[8];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int lv = 4 * q + j;
          float2 fp = make_float2(0.0f, 0.0f);
          if (valid && lv < F.levels) fp = load_feat2<P>(a.feat, (int64_t)lv * a.n_slots + sl);
          pos[2 * j] = fp.x;
          pos[2 * j + 1] = fp.y;
        }
        f3 W = {0.f, 0.f, 0.f};
        if (q == 0 && valid) W = {a.wr[sl], a.wg[sl], a.wb[sl]};
        const f32x4 out = mlp_forward16_f32(reinterpret_cast<const float *>(lds_w) + wofs,
                                            F.hidden, pos, dir, gin);
        if (q == 0 && valid) {
          S.x = fmaf(W.x, decode_lp(out[0], F.psi, F.kappa), S.x);
          S.y = fmaf(W.y, decode_lp(out[1], F.psi, F.kappa), S.y);
          S.z = fmaf(W.z, decode_lp(out[2], F.psi, F.kappa), S.z);
        }
      }
    } else {
      // 16-bit features are stored as the matrix-core operand expects them (level 4q+j in
      // 32-bit word j of lane group q), so loaded words become the B operand as they are
      typedef Mma<P> M;
      typedef typename M::vec vec;
      typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
      const uint32_t *fw = reinterpret_cast<const uint32_t *>(a.feat);
      u32x4 dw = {0u, 0u, 0u, 0u};
      if (cnt > 0) {
        const uint32_t *dfw = reinterpret_cast<const uint32_t *>(a.dfeat);
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (4 * q + k < F.levels) dw[k] = dfw[(int64_t)(4 * q + k) * a.n_entries + t];
      }
      const vec b1 = __builtin_bit_cast(vec, dw);
      float gz[8] = {gin, 0, 0, 0, 0, 0, 0, 0};
      const vec b2 = M::pack(gz);
      // the direction and g products of the input layer are the same for every query of a
      // column's ray: computed once per tile of rays
      f32x4 pre[4];
      mlp_input16<P>(reinterpret_cast<const vec *>(lds_w), b1, b2, pre);
      // the loads of query k+1 are issued before the network of query k runs
      auto load_k = [&](int k, u32x4 &pw, f3 &W) {
        pw = u32x4{0u, 0u, 0u, 0u};
        W = {0.f, 0.f, 0.f};
        if (k < cnt) {
          const int64_t sl = wf_slot(t, k);
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (4 * q + j < F.levels) pw[j] = fw[(int64_t)(4 * q + j) * a.n_slots + sl];
          if (q == 0) W = {a.wr[sl], a.wg[sl], a.wb[sl]};
        }
      };
      u32x4 pw;
      f3 W;
      load_k(0, pw, W);
      for (int k = 0; k < kmax; ++k) {
        int wofs = 0;  // opaque offset: keeps the LDS weight reads inside the loop
        asm volatile("" : "+s"(wofs));
        const u32x4 pc = pw;
        const f3 Wc = W;
        if (k + 1 < kmax) load_k(k + 1, pw, W);
        const f32x4 out = mlp_rest16<P>(reinterpret_cast<const vec *>(lds_w) + wofs, F.hidden,
                                        __builtin_bit_cast(vec, pc), pre);
        if (q == 0 && k < cnt) {
          S.x = fmaf(Wc.x, decode_lp(out[0], F.psi, F.kappa), S.x);
          S.y = fmaf(Wc.y, decode_lp(out[1], F.psi, F.kappa), S.y);
          S.z = fmaf(Wc.z, decode_lp(out[2], F.psi, F.kappa), S.z);
        }
      }
    }
    // continuing rays carry the sum to the next round; ended rays (also those without a query
    // this round) store it
    if (q == 0 && next != -2) {
      float *dst = next >= 0 ? a.out_ci + 3 * (size_t)next : a.acc_i + 3 * (size_t)r;
      dst[0] = ci.x + S.x;
      dst[1] = ci.y + S.y;
      dst[2] = ci.z + S.z;
    }
  }
}

// The field kernel for 8 features per level (4 feature groups): the same tiles and sums as
// wf_field_kernel; a lane loads 16 (FP32: 32) bytes per level and query, and word g of level
// 4q+j goes to word j of feature group g's operand.  Its larger weight image sets its occupancy.
// With 16-bit weights, workgroups of 8 waves share one copy of the weight image (about 70 KB
// with 5 hidden layers), so two resident workgroups give 4 waves per SIMD; the FP32 image, twice
// the size, keeps workgroups of 4 waves and the registers of one wave per SIMD.
template <int P>
constexpr int wf8_threads() { return P == P_F32 ? 256 : 512; }
template <int P>
__global__ __launch_bounds__(wf8_threads<P>())
__attribute__((amdgpu_waves_per_eu(P == P_F32 ? 1 : 4, 8))) void wf_field8_kernel(WfFieldArgs a) {
  extern __shared__ __align__(16) unsigned char lds_w[];
  stage_weights(lds_w, a.mlp, a.mlp_bytes);
  __syncthreads();
  constexpr int FG = 4;
  const FieldDev &F = *a.F;
  const int lane = lane_id(), q = lane >> 4, col = lane & 15;
  const int waves = (int)gridDim.x * (wf8_threads<P>() / 64);
  const int w0 = __builtin_amdgcn_readfirstlane((int)blockIdx.x * (wf8_threads<P>() / 64) +
                                                (int)(threadIdx.x >> 6));
  const int n_tiles = (a.n_entries + 15) >> 4;
  for (int rt = w0; rt < n_tiles; rt += waves) {
    const int t = rt * 16 + col;
    const bool tv = t < a.n_entries;
    const int cnt = tv ? a.ent_cnt[t] : 0;
    const int next = tv ? a.ent_next[t] : -2;
    int kmax = cnt;
#pragma unroll
    for (int o = 8; o >= 1; o >>= 1) kmax = max(kmax, __shfl_xor(kmax, o));
    kmax = __builtin_amdgcn_readfirstlane(kmax);
    uint32_t r = 0;
    f3 ci = {0.f, 0.f, 0.f};
    if (next != -2) {
      r = a.ent_ray[t];
      if (t < a.n_cont)
        ci = {a.in_ci[3 * (size_t)t], a.in_ci[3 * (size_t)t + 1], a.in_ci[3 * (size_t)t + 2]};
    }
    float gin = 0.0f;
    if (cnt > 0 && q == 0) gin = a.jobs[find_job_ray(a.jobs, a.n_jobs, (int64_t)r)].g;
    f3 S = {0.f, 0.f, 0.f};
    if constexpr (P == P_F32) {
      const float4 *df4 = reinterpret_cast<const float4 *>(a.dfeat);
      const float4 *pf4 = reinterpret_cast<const float4 *>(a.feat);
      float dir[FG][8];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float4 lo = make_float4(0.f, 0.f, 0.f, 0.f), hi = lo;
        const int lv = 4 * q + j;
        if (cnt > 0 && lv < F.levels) {
          const int64_t i = (int64_t)lv * a.n_entries + t;
          lo = df4[2 * i];
          hi = df4[2 * i + 1];
        }
        const float v[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
#pragma unroll
        for (int g = 0; g < FG; ++g) {
          dir[g][2 * j] = v[2 * g];
          dir[g][2 * j + 1] = v[2 * g + 1];
        }
      }
      for (int k = 0; k < kmax; ++k) {
        const bool valid = k < cnt;
        const int64_t sl = wf_slot(t, k);
        float pos[FG][8];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          float4 lo = make_float4(0.f, 0.f, 0.f, 0.f), hi = lo;
          const int lv = 4 * q + j;
          if (valid && lv < F.levels) {
            const int64_t i = (int64_t)lv * a.n_slots + sl;
            lo = pf4[2 * i];
            hi = pf4[2 * i + 1];
          }
          const float v[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
#pragma unroll
          for (int g = 0; g < FG; ++g) {
            pos[g][2 * j] = v[2 * g];
            pos[g][2 * j + 1] = v[2 * g + 1];
          }
        }
        f3 W = {0.f, 0.f, 0.f};
        if (q == 0 && valid) W = {a.wr[sl], a.wg[sl], a.wb[sl]};
        const f32x4 out = mlp_forward16_f32_g<FG>(reinterpret_cast<const float *>(lds_w),
                                                  F.hidden, pos, dir, gin);
        if (q == 0 && valid) {
          S.x = fmaf(W.x, decode_lp(out[0], F.psi, F.kappa), S.x);
          S.y = fmaf(W.y, decode_lp(out[1], F.psi, F.kappa), S.y);
          S.z = fmaf(W.z, decode_lp(out[2], F.psi, F.kappa), S.z);
        }
      }
    } else {
      typedef Mma<P> M;
      typedef typename M::vec vec;
      typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
      const uint4 *fw = reinterpret_cast<const uint4 *>(a.feat);
      const uint4 *dfw = reinterpret_cast<const uint4 *>(a.dfeat);
      u32x4 dwg[FG];
#pragma unroll
      for (int g = 0; g < FG; ++g) dwg[g] = u32x4{0u, 0u, 0u, 0u};
      if (cnt > 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (4 * q + j < F.levels) {
            const uint4 w4 = dfw[(int64_t)(4 * q + j) * a.n_entries + t];
            dwg[0][j] = w4.x;
            dwg[1][j] = w4.y;
            dwg[2][j] = w4.z;
            dwg[3][j] = w4.w;
          }
      }
      vec b1[FG];
#pragma unroll
      for (int g = 0; g < FG; ++g) b1[g] = __builtin_bit_cast(vec, dwg[g]);
      float gz[8] = {gin, 0, 0, 0, 0, 0, 0, 0};
      const vec *w = reinterpret_cast<const vec *>(lds_w);
      f32x4 pre[4];
      mlp_input16_g<P, FG>(w, b1, M::pack(gz), pre);
      // the loads of query k+1 are issued before the network of query k runs
      auto load_k = [&](int k, u32x4 (&pwg)[FG], f3 &W) {
#pragma unroll
        for (int g = 0; g < FG; ++g) pwg[g] = u32x4{0u, 0u, 0u, 0u};
        W = {0.f, 0.f, 0.f};
        if (k < cnt) {
          const int64_t sl = wf_slot(t, k);
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (4 * q + j < F.levels) {
              const uint4 w4 = fw[(int64_t)(4 * q + j) * a.n_slots + sl];
              pwg[0][j] = w4.x;
              pwg[1][j] = w4.y;
              pwg[2][j] = w4.z;
              pwg[3][j] = w4.w;
            }
          if (q == 0) W = {a.wr[sl], a.wg[sl], a.wb[sl]};
        }
      };
      u32x4 pwg[FG];
      f3 W;
      load_k(0, pwg, W);
      for (int k = 0; k < kmax; ++k) {
        int wofs = 0;  // opaque offset: keeps the LDS weight reads inside the loop
        asm volatile("" : "+s"(wofs));
        vec b0[FG];
#pragma unroll
        for (int g = 0; g < FG; ++g) b0[g] = __builtin_bit_cast(vec, pwg[g]);
        const f3 Wc = W;
        if (k + 1 < kmax) load_k(k + 1, pwg, W);
        const f32x4 out = mlp_rest16_g<P, FG>(w + wofs, F.hidden, b0, pre);
        if (q == 0 && k < cnt) {
          S.x = fmaf(Wc.x, decode_lp(out[0], F.psi, F.kappa), S.x);
          S.y = fmaf(Wc.y, decode_lp(out[1], F.psi, F.kappa), S.y);
          S.z = fmaf(Wc.z, decode_lp(out[2], F.psi, F.kappa), S.z);
        }
      }
    }
    if (q == 0 && next != -2) {
      float *dst = next >= 0 ? a.out_ci + 3 * (size_t)next : a.acc_i + 3 * (size_t)r;
      dst[0] = ci.x + S.x;
      dst[1] = ci.y + S.y;
      dst[2] = ci.z + S.z;
    }
  }
}

__global__ void wf_resolve_kernel(WfResolveArgs a) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.pix_begin[a.n_jobs]) return;
  int lo = 0, hi = a.n_jobs - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (a.pix_begin[mid] <= p) lo = mid;
    else hi = mid - 1;
  }
  const MarchJob &job = a.jobs[lo];
  const int pi = (int)(p - a.pix_begin[lo]);
  const int x = pi % job.width, y = pi / job.width;
  const int tile = (y / a.tile_h) * job.tiles_x + x / a.tile_w;
  const int ln = (y % a.tile_h) * a.tile_w + x % a.tile_w;
  const int64_t per_s = (int64_t)job.tiles * 64;
  f3 C = {0.f, 0.f, 0.f};
  for (int s = 0; s < job.spp; ++s) {
    const size_t r = (size_t)(job.ray_begin + s * per_s + tile * 64 + ln) * 3;
    C = C + (f3{a.acc_d[r], a.acc_d[r + 1], a.acc_d[r + 2]} +
             f3{a.acc_i[r], a.acc_i[r + 1], a.acc_i[r + 2]});
  }
  float *o = job.out + (size_t)pi * 3;
  o[0] = C.x * job.inv_spp;
  o[1] = C.y * job.inv_spp;
  o[2] = C.z * job.inv_spp;
}

// ------------------------------------------------------------------ host side
template <typename T>
static hipError_t alloc_n(T *&p, size_t n) {
  return hipMalloc((void **)&p, sizeof(T) * n);
}

template <typename T>
static void free_p(T *&p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

static void free_entries(WfState &w) {
  for (int i = 0; i < 2; ++i) {
    free_p(w.list_ray[i]);
    free_p(w.list_j[i]);
    free_p(w.list_T[i]);
    free_p(w.list_cd[i]);
    free_p(w.list_ci[i]);
    WfRound &b = w.rb[i];
    free_p(b.ent_ray);
    free_p(b.ent_cnt);
    free_p(b.ent_next);
    free_p(b.ent_u);
    free_p(b.ent_mask);
    for (int k = 0; k < 6; ++k) free_p(b.slot[k]);
    free_p(b.feat);
    free_p(b.dfeat);
  }
  w.ent_cap = 0;
  w.feat_elem = 0;
}

hipError_t wf_reserve(WfState &w, size_t entries, size_t rays, size_t feat_bytes) {
  hipError_t e = hipSuccess;
  if (entries > w.ent_cap || feat_bytes > w.feat_elem) {
    free_entries(w);
    const size_t slots = (size_t)wf_slots((int64_t)entries);
    for (int i = 0; i < 2; ++i) {
      if ((e = alloc_n(w.list_ray[i], entries))) return e;
      if ((e = alloc_n(w.list_j[i], entries))) return e;
      if ((e = alloc_n(w.list_T[i], entries))) return e;
      if ((e = alloc_n(w.list_cd[i], entries * 3))) return e;
      if ((e = alloc_n(w.list_ci[i], entries * 3))) return e;
      WfRound &b = w.rb[i];
      if ((e = alloc_n(b.ent_ray, entries))) return e;
      if ((e = alloc_n(b.ent_cnt, entries))) return e;
      if ((e = alloc_n(b.ent_next, entries))) return e;
      if ((e = alloc_n(b.ent_u, entries))) return e;
      if ((e = alloc_n(b.ent_mask, entries))) return e;
      for (int k = 0; k < 6; ++k)
        if ((e = alloc_n(b.slot[k], slots))) return e;
      unsigned char *fp = nullptr;
      if ((e = alloc_n(fp, slots * PFN_MAX_LEVELS * feat_bytes))) return e;
      b.feat = fp;
      fp = nullptr;
      if ((e = alloc_n(fp, entries * PFN_MAX_LEVELS * feat_bytes))) return e;
      b.dfeat = fp;
    }
    w.ent_cap = entries;
    w.feat_elem = feat_bytes;
  }
  if (rays * 3 > w.acc_cap) {
    free_p(w.acc_d);
    free_p(w.acc_i);
    w.acc_cap = 0;
    if ((e = alloc_n(w.acc_d, rays * 3))) return e;
    if ((e = alloc_n(w.acc_i, rays * 3))) return e;
    w.acc_cap = rays * 3;
  }
  for (int i = 0; i < 2; ++i)
    if (!w.rb[i].count && (e = hipMalloc((void **)&w.rb[i].count, 16))) return e;
  if (!w.host_count && (e = hipHostMalloc((void **)&w.host_count, 16, hipHostMallocDefault)))
    return e;
  if (!w.side) {
    // default priority, and not synchronising with the null stream
    if ((e = hipStreamCreateWithFlags(&w.side, hipStreamNonBlocking))) return e;
    if ((e = hipStreamCreateWithFlags(&w.side2, hipStreamNonBlocking))) return e;
    for (int i = 0; i < 2; ++i) {
      if ((e = hipEventCreateWithFlags(&w.ev_march[i], hipEventDisableTiming))) return e;
      if ((e = hipEventCreateWithFlags(&w.ev_field[i], hipEventDisableTiming))) return e;
      if ((e = hipEventCreateWithFlags(&w.ev_enc[i], hipEventDisableTiming))) return e;
    }
    if ((e = hipEventCreateWithFlags(&w.ev_done, hipEventDisableTiming))) return e;
  }
  return hipSuccess;
}

void wf_release(WfState &w) {
  if (w.side) (void)hipStreamSynchronize(w.side);
  if (w.side2) (void)hipStreamSynchronize(w.side2);
  free_entries(w);
  free_p(w.acc_d);
  free_p(w.acc_i);
  for (int i = 0; i < 2; ++i) free_p(w.rb[i].count);
  if (w.host_count) (void)hipHostFree(w.host_count);
  free_p(w.pix_begin);
  for (int i = 0; i < 2; ++i) {
    if (w.ev_march[i]) (void)hipEventDestroy(w.ev_march[i]);
    if (w.ev_field[i]) (void)hipEventDestroy(w.ev_field[i]);
    if (w.ev_enc[i]) (void)hipEventDestroy(w.ev_enc[i]);
  }
  if (w.ev_done) (void)hipEventDestroy(w.ev_done);
  if (w.side) (void)hipStreamDestroy(w.side);
  if (w.side2) (void)hipStreamDestroy(w.side2);
  w = WfState{};
}

template <typename VT, int DIRECT>
static void launch_k1(const WfArgs &a, int blocks, hipStream_t st) {
  hipLaunchKernelGGL((wf_march_kernel<VT, DIRECT>), dim3(blocks), dim3(WF_THREADS), 0, st, a);
}

template <int P, int FG>
static hipError_t launch_k23(pfn_context *ctx, hipStream_t st, const WfEncArgs &e,
                             const WfDirArgs &dg, const std::vector<std::pair<int, int>> &groups,
                             const WfFieldArgs &f, int field_blocks, bool split_levels,
                             hipStream_t fst, hipEvent_t enc_done) {
  // the direction encoding only needs the march kernel's outputs: with a field stream it runs
  // there, beside the position encodings
  {
    hipStream_t ds = fst ? fst : st;
    const int ts = timing_begin_on(ctx, ds);
    hipLaunchKernelGGL((wf_dir_kernel<P, FG>), dim3((dg.n_entries + WF_THREADS - 1) / WF_THREADS),
                       dim3(WF_THREADS), 0, ds, dg);
    timing_end_on(ctx, ts, TK_WF_DIR, ds);
  }
  const int64_t threads = (((int64_t)e.n_entries + 63) >> 6) << (6 + e.kshift);
  for (auto &g : groups) {
    WfEncArgs ee = e;
    ee.l0 = g.first;
    ee.l1 = g.second;
    // fine levels spread over the XCDs are marked by a negative end: -(level count)
    // all levels paired over the XCDs in one launch are marked by a negative start
    ee.paired = g.first < 0 ? 1 : 0;
    if (ee.paired) ee.l0 = 0;
    ee.xcd_levels = !ee.paired && g.second < 0 ? -g.second : 0;
    if (ee.xcd_levels) ee.l1 = g.first + ee.xcd_levels;
    ee.per_level = !ee.paired && !ee.xcd_levels && split_levels && g.second - g.first > 1
                       ? (int)threads
                       : 0;
    const int64_t n = ee.per_level ? threads * (g.second - g.first) : threads;
    int eb = (int)((n + WF_THREADS - 1) / WF_THREADS);
    if (ee.paired) {
      eb *= 8;
    } else if (ee.xcd_levels) {
      const int per = 8 / ee.xcd_levels;
      eb = 8 * ((eb + per - 1) / per);
    }
    const int ts = timing_begin_on(ctx, st);
    hipLaunchKernelGGL((wf_encode_kernel<P, FG>), dim3(eb), dim3(WF_THREADS), 0, st, ee);
    timing_end_on(ctx, ts, TK_WF_ENCODE, st);
  }
  if (fst) {
    hipError_t err = hipEventRecord(enc_done, st);
    if (err == hipSuccess) err = hipStreamWaitEvent(fst, enc_done, 0);
    if (err != hipSuccess) return err;
    st = fst;
  }
  const int ts = timing_begin_on(ctx, st);
  if constexpr (FG == 1)
    hipLaunchKernelGGL((wf_field_kernel<P>), dim3(field_blocks), dim3(WF_THREADS),
                       (size_t)f.mlp_bytes, st, f);
  else
    hipLaunchKernelGGL((wf_field8_kernel<P>), dim3(field_blocks), dim3(wf8_threads<P>()),
                       (size_t)f.mlp_bytes, st, f);
  timing_end_on(ctx, ts, TK_WF_FIELD, st);
  return hipSuccess;
}

hipError_t wf_launch_field_pass(pfn_context *ctx, hipStream_t st, int prec, const WfEncArgs &e,
                                const WfDirArgs &dg, const std::vector<std::pair<int, int>> &groups,
                                const WfFieldArgs &f, int field_blocks, bool split_levels,
                                hipStream_t field_st, hipEvent_t enc_done) {
  if (f.fg != 1) {
    if (prec == P_F32)
      return launch_k23<P_F32, 4>(ctx, st, e, dg, groups, f, field_blocks, split_levels, field_st,
                                  enc_done);
    if (prec == P_BF16)
      return launch_k23<P_BF16, 4>(ctx, st, e, dg, groups, f, field_blocks, split_levels,
                                   field_st, enc_done);
    return launch_k23<P_F16, 4>(ctx, st, e, dg, groups, f, field_blocks, split_levels, field_st,
                                enc_done);
  }
  if (prec == P_F32)
    return launch_k23<P_F32, 1>(ctx, st, e, dg, groups, f, field_blocks, split_levels, field_st,
                                enc_done);
  if (prec == P_BF16)
    return launch_k23<P_BF16, 1>(ctx, st, e, dg, groups, f, field_blocks, split_levels, field_st,
                                 enc_done);
  return launch_k23<P_F16, 1>(ctx, st, e, dg, groups, f, field_blocks, split_levels, field_st,
                              enc_done);
}

template <int P>
static int field_blocks_resident(int mlp_bytes, int fg) {
  int per_cu = 0;
  const hipError_t e =
      fg == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, wf_field_kernel<P>,
                                                             WF_THREADS, (size_t)mlp_bytes)
              : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, wf_field8_kernel<P>,
                                                             wf8_threads<P>(), (size_t)mlp_bytes);
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  int cus = 256;
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return per_cu * cus;
}

int wf_field_blocks(int prec, int mlp_bytes, int fg) {
  return prec == P_F32    ? field_blocks_resident<P_F32>(mlp_bytes, fg)
         : prec == P_BF16 ? field_blocks_resident<P_BF16>(mlp_bytes, fg)
                          : field_blocks_resident<P_F16>(mlp_bytes, fg);
}

std::vector<std::pair<int, int>> wf_level_groups(const pfn_context *ctx, int slot,
                                                 const FieldDev &fd_host, size_t fbytes) {
  std::vector<std::pair<int, int>> groups;
  const FieldSlot &fs = ctx->fields[slot];
  const int L = fd_host.levels;
  auto fine = [&](int l) {
    return !((fd_host.pos.dense_mask >> l) & 1u) && fd_host.pos.res[l] >= WF_FINE_RES;
  };
  auto bytes = [&](int l) {
    const size_t end = l + 1 < L ? fd_host.pos.off[l + 1] : fs.pos_entries;
    return (end - fd_host.pos.off[l]) * fbytes;
  };
  int l = 0;
  while (l < L) {
    int e = l + 1;
    if (!fine(l)) {
      size_t b = bytes(l);
      while (e < L && !fine(e) && b + bytes(e) <= WF_GROUP_BYTES) b += bytes(e++);
    }
    groups.push_back({l, e});
    l = e;
  }
  return groups;
}

void wf_launch_resolve(pfn_context *ctx, hipStream_t st, const WfResolveArgs &ra, int64_t pixels) {
  const int ts = timing_begin_on(ctx, st);
  hipLaunchKernelGGL(wf_resolve_kernel, dim3((unsigned)((pixels + 255) / 256)), dim3(256), 0, st,
                     ra);
  timing_end_on(ctx, ts, TK_WF_RESOLVE, st);
}

// Rounds of the wavefront render.  The march kernel of round r runs on the context's stream;
// the encoding kernels of round r run on a side stream once the march kernel has finished, and
// its field kernel on a second side stream once they have, while the march kernel of round r+1
// (which only needs the list of continuing rays) already runs on the context's stream and the
// encodings of round r+1 may run beside the field kernel of round r.  Round r+2 reuses round
// r's buffers, so its march kernel waits for round r's field kernel.  The field kernels follow
// one another on their stream (each reads the indirect sums the previous one carried).  With
// `overlap` off the side streams are not used.
pfn_status run_wavefront(pfn_context *ctx, const MarchArgs &m, std::vector<MarchJob> &mj,
                         int direct, int prec, int slot, const FieldDev &fd_host, bool overlap) {
  WfState &w = ctx->wf;
  // ray layout and pixel offsets of the jobs
  int64_t rays = 0, pixels = 0;
  std::vector<int64_t> pix_begin(mj.size() + 1);
  for (size_t i = 0; i < mj.size(); ++i) {
    mj[i].ray_begin = rays;
    rays += (int64_t)mj[i].spp * mj[i].tiles * 64;
    pix_begin[i] = pixels;
    pixels += (int64_t)mj[i].width * mj[i].height;
  }
  pix_begin[mj.size()] = pixels;
  if (rays >= (int64_t)1 << 31)
    return pfn_fail(ctx, PFN_ERR_UNSUPPORTED, "wavefront render: more than 2^31 ray samples");
  // rounds of fewer rays for wider features, so that the feature buffers keep their size
  const int fg = fd_host.fg;
  const size_t entries = (size_t)std::min<int64_t>(rays, WF_MAX_ENTRIES / fg);
  const size_t fbytes = (prec == P_F32 ? 8 : 4) * (size_t)fg;
  PFN_HIP(ctx, wf_reserve(w, entries, (size_t)rays, fbytes));
  if (w.pix_cap < mj.size() + 1) {
    free_p(w.pix_begin);
    w.pix_cap = 0;
    PFN_HIP(ctx, hipMalloc((void **)&w.pix_begin, sizeof(int64_t) * (mj.size() + 1)));
    w.pix_cap = mj.size() + 1;
  }
  PFN_HIP(ctx, hipMemcpyAsync(ctx->jobs_dev, mj.data(), sizeof(MarchJob) * mj.size(),
                              hipMemcpyHostToDevice, ctx->stream));
  PFN_HIP(ctx, hipMemcpyAsync(w.pix_begin, pix_begin.data(), sizeof(int64_t) * pix_begin.size(),
                              hipMemcpyHostToDevice, ctx->stream));
  PFN_HIP(ctx, hipStreamSynchronize(ctx->stream));

  std::vector<std::pair<int, int>> groups;
  if (fg > 1 && fd_host.levels >= 8) {
    // 8 features per level: a hashed level's table is 4x the 2-feature one (8 MB at 2^19
    // entries), two of them no longer share an XCD's L2 well; launches of up to 8 levels, one
    // per XCD (measured on a 1080p frame, 16 levels at growth 2: 108 against 121 ms per frame
    // with the levels paired).  Runs of 8, 4, 2, 1 levels, marked by the end -(level count).
    for (int l = 0, left = fd_host.levels; left > 0;) {
      const int take = left >= 8 ? 8 : left >= 4 ? 4 : left >= 2 ? 2 : 1;
      groups.push_back({l, -take});
      l += take;
      left -= take;
    }
  } else if (fd_host.levels >= 8 && fd_host.levels <= 16) {
    // one launch, the levels paired over the XCDs; marked by a negative start
    groups.push_back({-1, fd_host.levels});
  } else {
    // runs of single fine levels go WF_XCD_LEVELS (then 2) at a time, each level on its own
    // share of the XCDs; marked by the end -(level count)
    const std::vector<std::pair<int, int>> g0 = wf_level_groups(ctx, slot, fd_host, fbytes);
    auto fine_single = [&](size_t i) {
      return g0[i].second == g0[i].first + 1 &&
             (fd_host.pos.dense_mask >> g0[i].first & 1u) == 0 &&
             fd_host.pos.res[g0[i].first] >= WF_FINE_RES;
    };
    for (size_t i = 0; i < g0.size();) {
      size_t run = 0;
      while (i + run < g0.size() && fine_single(i + run)) ++run;
      if (run == 0) {
        groups.push_back(g0[i++]);
        continue;
      }
      while (run > 0) {
        const int take = run >= WF_XCD_LEVELS ? WF_XCD_LEVELS : run >= 2 ? 2 : 1;
        groups.push_back(take == 1 ? g0[i] : std::make_pair(g0[i].first, -take));
        i += take;
        run -= take;
      }
    }
  }
  const int fb_max = wf_field_blocks(prec, m.mlp_bytes, fg);
  // march kernels on sa, encodings on sb, field kernels on sc
  hipStream_t sa = ctx->stream, sb = overlap ? w.side : ctx->stream,
              sc = overlap ? w.side2 : ctx->stream;

  const int tslot = timing_begin(ctx);
  int64_t fresh_next = 0;
  int n_cont = 0, cur = 0;
  for (int r = 0; fresh_next < rays || n_cont > 0; ++r) {
    const int p = r & 1;
    WfRound &b = w.rb[p];
    const int n_fresh = (int)std::min<int64_t>((int64_t)entries - n_cont, rays - fresh_next);
    const int n_in = n_cont + n_fresh;

    WfArgs a{};
    a.m = m;
    a.in = {w.list_ray[cur], w.list_j[cur], w.list_T[cur], w.list_cd[cur], w.list_ci[cur]};
    a.out = {w.list_ray[cur ^ 1], w.list_j[cur ^ 1], w.list_T[cur ^ 1], w.list_cd[cur ^ 1],
             w.list_ci[cur ^ 1]};
    a.n_cont = n_cont;
    a.n_fresh = n_fresh;
    a.fresh_begin = fresh_next;
    a.out_count = b.count;
    a.ent_ray = b.ent_ray;
    a.ent_cnt = b.ent_cnt;
    a.ent_next = b.ent_next;
    a.ent_u = b.ent_u;
    a.qx = b.slot[0];
    a.qy = b.slot[1];
    a.qz = b.slot[2];
    a.wr = b.slot[3];
    a.wg = b.slot[4];
    a.wb = b.slot[5];
    a.acc_d = w.acc_d;
    a.acc_i = w.acc_i;

    // march kernel of round r: its buffers were last read by round r-2's field kernel
    if (overlap && r >= 2) PFN_HIP(ctx, hipStreamWaitEvent(sa, w.ev_field[p], 0));
    PFN_HIP(ctx, hipMemsetAsync(b.count, 0, 4, sa));
    const int needed = (n_in + WF_THREADS - 1) / WF_THREADS;
    const int k1_blocks = ((needed + 7) / 8) * 8;
    const int ts1 = timing_begin_on(ctx, sa);
    if (ctx->vol_dtype == PFN_F16) {
      if (direct == PFN_DIRECT_LIGHT_VOLUME) launch_k1<__half, PFN_DIRECT_LIGHT_VOLUME>(a, k1_blocks, sa);
      else launch_k1<__half, PFN_DIRECT_SHADOW_RAYS>(a, k1_blocks, sa);
    } else {
      if (direct == PFN_DIRECT_LIGHT_VOLUME) launch_k1<float, PFN_DIRECT_LIGHT_VOLUME>(a, k1_blocks, sa);
      else launch_k1<float, PFN_DIRECT_SHADOW_RAYS>(a, k1_blocks, sa);
    }
    timing_end_on(ctx, ts1, TK_WF_MARCH, sa);
    PFN_HIP(ctx, hipGetLastError());
    PFN_HIP(ctx, hipMemcpyAsync(w.host_count + p, b.count, 4, hipMemcpyDeviceToHost, sa));
    PFN_HIP(ctx, hipEventRecord(w.ev_march[p], sa));

    // encoding and field kernels of round r
    WfEncArgs e{};
    e.F = m.fields + slot;
    e.ent_cnt = b.ent_cnt;
    e.qx = b.slot[0];
    e.qy = b.slot[1];
    e.qz = b.slot[2];
    e.feat = b.feat;
    e.n_slots = wf_slots(n_in);
    e.n_entries = n_in;
    e.kshift = WF_SLOTS_LOG2;
    WfDirArgs dg{};
    dg.F = m.fields + slot;
    dg.ent_cnt = b.ent_cnt;
    dg.ent_u = b.ent_u;
    dg.dfeat = b.dfeat;
    dg.n_entries = n_in;
    WfFieldArgs f{};
    f.F = m.fields + slot;
    f.mlp = ctx->fields[slot].mlp_packed[prec];
    f.mlp_bytes = m.mlp_bytes;
    f.jobs = m.jobs;
    f.n_jobs = m.n_jobs;
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
    f.n_entries = n_in;
    f.n_cont = n_cont;
    f.fg = fg;
    f.in_ci = w.list_ci[cur];
    f.out_ci = w.list_ci[cur ^ 1];
    const int fb = std::max(1, std::min((n_in + 63) / 64, fb_max));
    if (overlap) {
      PFN_HIP(ctx, hipStreamWaitEvent(sb, w.ev_march[p], 0));
      PFN_HIP(ctx, hipStreamWaitEvent(sc, w.ev_march[p], 0));
    }
    PFN_HIP(ctx, wf_launch_field_pass(ctx, sb, prec, e, dg, groups, f, fb, false,
                                      overlap ? w.side2 : nullptr, w.ev_enc[p]));
    PFN_HIP(ctx, hipGetLastError());
    PFN_HIP(ctx, hipEventRecord(w.ev_field[p], sc));

    // the next round needs the number of continuing rays
    PFN_HIP(ctx, hipEventSynchronize(w.ev_march[p]));
    fresh_next += n_fresh;
    n_cont = (int)w.host_count[p];
    cur ^= 1;
  }
  // the resolve reads every ray's final sums: after the last field kernel
  if (overlap) {
    PFN_HIP(ctx, hipEventRecord(w.ev_done, sc));
    PFN_HIP(ctx, hipStreamWaitEvent(sa, w.ev_done, 0));
  }
  WfResolveArgs ra{};
  ra.jobs = m.jobs;
  ra.n_jobs = m.n_jobs;
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
