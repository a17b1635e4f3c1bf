// Ray marcher with direct light and indirect light from the photon field, the photon cache or
// nothing (Section 3.6: the field replaces the multiple-scattering term of a ray marcher;
// Eq. (3): L = L_d + L_i).  One lane marches one ray; a wave owns a 64-pixel tile; a workgroup
// of 4 waves owns a block of 4 tiles of one job, so a batch of uneven frames is one launch.
//
// Per step: brick-ordered trilinear density, transfer function from LDS, alpha from the
// extinction, direct light (shadow march or light-transmittance volume) and front-to-back
// compositing.  With the field, the wave runs in groups of `stride` steps: each lane keeps the
// query position of its group's first step and the group weight W = sum T*alpha*albedo, and
// after the group the whole wave evaluates the field for its 64 queries on the matrix cores and
// adds W * L_i (sample-and-hold of the field value over the group, exact by linearity).
#include "march.h"
#include "march_dev.h"
#include "pfn_ctx.h"

#define MARCH_THREADS 256

// Field evaluation for the 64 queries of a wave (one per lane); returns the decoded L_i of this
// lane's own query.  Must be called by all 64 lanes.
template <int P>
__device__ f3 field_eval_wave(const FieldDev &F, const void *lds_w, f3 xq, float u0, float u1,
                              float g, bool valid) {
  const int lane = lane_id();
  const uint64_t vm = ballot(valid);
  float r0 = 0.f, r1 = 0.f, r2 = 0.f;
#pragma unroll 1
  for (int j = 0; j < 4; ++j) {
    if (((vm >> (16 * j)) & 0xFFFFull) == 0) continue;
    const int src = 16 * j + (lane & 15);
    f3 x = {__shfl(xq.x, src), __shfl(xq.y, src), __shfl(xq.z, src)};
    float a0 = __shfl(u0, src), a1 = __shfl(u1, src);
    bool v = (vm >> src) & 1ull;
    f32x4 out = field_tile16<P>(F, lds_w, x, a0, a1, g, v);
    float o0 = __shfl(out[0], lane & 15), o1 = __shfl(out[1], lane & 15),
          o2 = __shfl(out[2], lane & 15);
    if ((lane >> 4) == j) {
      r0 = o0;
      r1 = o1;
      r2 = o2;
    }
  }
  if (!valid) return {0.f, 0.f, 0.f};
  return {decode_lp(r0, F.psi, F.kappa), decode_lp(r1, F.psi, F.kappa),
          decode_lp(r2, F.psi, F.kappa)};
}

// Job of logical block b: the last job whose first block is <= b.
__device__ __forceinline__ int find_job(const MarchArgs &a, int b) {
  int lo = 0, hi = a.n_jobs - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (a.jobs[mid].block_begin <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Pop the next logical block from the per-XCD queues: XCD x owns the contiguous block range
// [x*per, (x+1)*per) so that neighbouring image blocks share that XCD's L2; a workgroup whose
// own queue is empty takes work from the others.  Returns -1 when every queue is empty, which
// every workgroup reaches after at most 8 failed pops.
__device__ __forceinline__ int pop_block(unsigned *queues, int xcd, int nb) {
  const int per = (nb + 7) >> 3;
  for (int k = 0; k < 8; ++k) {
    const int x = (xcd + k) & 7;
    const int begin = x * per;
    const int size = min(per, nb - begin);
    if (size <= 0) continue;
    unsigned v = atomicAdd(&queues[x], 1u);
    if (v < (unsigned)size) return begin + (int)v;
  }
  return -1;
}

// One block of 4 wave tiles of one job.
template <typename VT, int DIRECT, int IND, int P>
__device__ __forceinline__ void march_block(const MarchArgs &a, const MarchJob &job, int b,
                                            const float4 *tf, const FieldDev &F,
                                            const void *lds_w) {
  // F refers to the job's field descriptor in global memory: the encoder indexes its per-level
  // arrays with lane-dependent levels, which a private copy would have to keep in scratch.
  const int lane = lane_id();
  const int wave = threadIdx.x >> 6;
  const int lb = b - job.block_begin;
  const int bx = lb % job.blocks_x, by = lb / job.blocks_x;
  const int px = bx * (a.tile_w * a.block_w) + (wave % a.block_w) * a.tile_w + lane % a.tile_w;
  const int py = by * (a.tile_h * a.block_h) + (wave / a.block_w) * a.tile_h + lane / a.tile_w;
  bool active = px < job.width && py < job.height;

  const f3 eye = {job.eye[0], job.eye[1], job.eye[2]};
  const f3 fw = {job.fwd[0], job.fwd[1], job.fwd[2]};
  const f3 rt = {job.right[0], job.right[1], job.right[2]};
  const f3 up = {job.up[0], job.up[1], job.up[2]};

  f3 C = {0.f, 0.f, 0.f};   // pixel sum over samples
  f3 Cs = {0.f, 0.f, 0.f};  // current sample
  int s = 0;
  bool live = false;
  f3 d = {0.f, 0.f, 1.f}, wo = {0.f, 0.f, -1.f};
  float t0 = 0.f, span = 0.f, xi = 0.5f, T = 1.0f, u0 = 0.f, u1 = 0.f;
  int n = 0, j = 0;
  f3 q = {0.f, 0.f, 0.f};
  unsigned n_steps = 0, n_queries = 0;
  const int group = (IND == PFN_INDIRECT_FIELD) ? job.stride : 0x7fffffff;

  for (;;) {
    // lanes without a live ray start their next sample (rays that miss add nothing)
    while (active && !live) {
      if (s == job.spp) {
        float *o = job.out + ((size_t)py * job.width + px) * 3;
        o[0] = C.x * job.inv_spp;
        o[1] = C.y * job.inv_spp;
        o[2] = C.z * job.inv_spp;
        active = false;
        if (a.counters) {
          atomicAdd(&a.counters[0], (unsigned long long)n_steps);
          atomicAdd(&a.counters[1], (unsigned long long)n_queries);
        }
        break;
      }
      float jx = 0.5f, jy = 0.5f;
      xi = 0.5f;
      if (job.spp > 1) {
        Philox r;
        r.init(job.seed, ((uint64_t)py * job.width + px) * (uint64_t)job.spp + (uint64_t)s,
               STREAM_RENDER);
        jx = r.next();
        jy = r.next();
        xi = r.next();
      }
      ++s;
      float sx = 2.0f * ((float)px + jx) / (float)job.width - 1.0f;
      float sy = 1.0f - 2.0f * ((float)py + jy) / (float)job.height;
      d = normalize3(fw + rt * sx + up * sy);
      wo = d * -1.0f;
      float t1;
      if (!clip_cube(eye, d, t0, t1)) continue;
      span = t1 - t0;
      float ns = ceilf(span / job.step);
      n = ns > (float)job.max_steps ? job.max_steps : (int)ns;
      j = 0;
      T = 1.0f;
      Cs = {0.f, 0.f, 0.f};
      if constexpr (IND == PFN_INDIRECT_FIELD) dir_coords(wo, u0, u1);
      live = n > 0;
    }
    if constexpr (IND == PFN_INDIRECT_FIELD) {
      if (ballot(active) == 0) break;
    } else {
      if (!active) break;
    }

    // one group of steps
    f3 W = {0.f, 0.f, 0.f};
    f3 xq = {0.f, 0.f, 0.f};
    bool finished = false;
    if (live) {
      for (int k = 0; k < group; ++k) {
        float l = fminf(job.step, span - (float)j * job.step);
        if (!(l > 0.0f)) {
          finished = true;
          break;
        }
        float t = t0 + (float)j * job.step + xi * l;
        f3 x = eye + d * t;
        float rho = density_march(reinterpret_cast<const VT *>(a.vol), a.vg, a.qvol, a.qg, x);
        float4 o = tf_lookup(tf, rho);
        float sig = o.w * a.ext_scale;
        float alpha = -expm1f(-sig * l);
        float att = 1.0f - alpha;
        f3 alb = {o.x, o.y, o.z};
        f3 Ld = direct_light<VT, DIRECT>(a, job, tf, x, wo);
        f3 wgt = alb * (T * alpha);
        ++n_steps;
        if constexpr (IND == PFN_INDIRECT_CACHE) {
          if (j % job.stride == 0) {
            q = cache_gather(a, job, x);
            ++n_queries;
          }
          Cs = Cs + mul(wgt, Ld + q);
        } else if constexpr (IND == PFN_INDIRECT_FIELD) {
          if (k == 0) xq = x;
          Cs = Cs + mul(wgt, Ld);
          W = W + wgt;
        } else {
          Cs = Cs + mul(wgt, Ld);
        }
        T *= att;
        ++j;
        if (j >= n || T < job.t_min) {
          finished = true;
          break;
        }
      }
    }
    if constexpr (IND == PFN_INDIRECT_FIELD) {
      bool valid = live && (W.x != 0.f || W.y != 0.f || W.z != 0.f);
      n_queries += valid ? 1u : 0u;
      if (ballot(valid) != 0) {
        f3 Li = field_eval_wave<P>(F, lds_w, xq, u0, u1, job.g, valid);
        Cs = Cs + mul(W, Li);
      }
    }
    if (live && finished) {
      C = C + Cs;
      live = false;
    }
  }
}

template <typename VT, int DIRECT, int IND, int P>
__global__ __launch_bounds__(MARCH_THREADS) void march_kernel(MarchArgs a) {
  __shared__ float4 tf[256];
  __shared__ int s_block;
  extern __shared__ __align__(16) unsigned char lds_w[];
  for (int i = threadIdx.x; i < 256; i += blockDim.x) tf[i] = a.tf[i];
  const int nb = a.total_blocks;
  if (!a.persistent) {
    // XCD-aware block order: the hardware deals workgroups round-robin to the 8 XCDs, so give
    // each XCD a contiguous run of logical blocks.
    const int per = (nb + 7) >> 3;
    const int b = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    if (b >= nb) return;
    const MarchJob job = a.jobs[find_job(a, b)];
    if constexpr (IND == PFN_INDIRECT_FIELD) stage_weights(lds_w, a.mlp[job.slot], a.mlp_bytes);
    __syncthreads();
    march_block<VT, DIRECT, IND, P>(a, job, b, tf, a.fields[job.slot], lds_w);
    return;
  }
  // persistent: workgroups pull blocks from the queues until all are empty
  int staged = -1;
  const int xcd = (int)(blockIdx.x & 7);
  for (;;) {
    if (threadIdx.x == 0) s_block = pop_block(a.queues, xcd, nb);
    __syncthreads();
    const int b = s_block;
    if (b < 0) break;
    const MarchJob job = a.jobs[find_job(a, b)];
    if constexpr (IND == PFN_INDIRECT_FIELD) {
      if (job.slot != staged) {
        stage_weights(lds_w, a.mlp[job.slot], a.mlp_bytes);
        staged = job.slot;
      }
    }
    __syncthreads();
    march_block<VT, DIRECT, IND, P>(a, job, b, tf, a.fields[job.slot], lds_w);
    __syncthreads();  // all waves are done with s_block and the staged weights
  }
}

__global__ void reset_queues_kernel(unsigned *q) {
  if (threadIdx.x < 8) q[threadIdx.x] = 0u;
}

// ------------------------------------------------------------------ host side
template <typename VT, int DIRECT, int IND, int P>
static hipError_t launch_t(const MarchArgs &a, int blocks, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL((march_kernel<VT, DIRECT, IND, P>), dim3(blocks), dim3(MARCH_THREADS), lds,
                     st, a);
  return hipGetLastError();
}

template <typename VT, int DIRECT, int IND>
static hipError_t launch_p(const MarchArgs &a, int prec, int blocks, size_t lds, hipStream_t st) {
  if constexpr (IND == PFN_INDIRECT_FIELD) {
    if (prec == P_F32) return launch_t<VT, DIRECT, IND, P_F32>(a, blocks, lds, st);
    if (prec == P_BF16) return launch_t<VT, DIRECT, IND, P_BF16>(a, blocks, lds, st);
    return launch_t<VT, DIRECT, IND, P_F16>(a, blocks, lds, st);
  } else {
    return launch_t<VT, DIRECT, IND, P_F16>(a, blocks, lds, st);
  }
}

template <typename VT, int DIRECT>
static hipError_t launch_i(const MarchArgs &a, int ind, int prec, int blocks, size_t lds,
                           hipStream_t st) {
  if (ind == PFN_INDIRECT_FIELD) return launch_p<VT, DIRECT, PFN_INDIRECT_FIELD>(a, prec, blocks, lds, st);
  if (ind == PFN_INDIRECT_CACHE) return launch_p<VT, DIRECT, PFN_INDIRECT_CACHE>(a, prec, blocks, lds, st);
  return launch_p<VT, DIRECT, PFN_INDIRECT_NONE>(a, prec, blocks, lds, st);
}

template <typename VT>
static hipError_t launch_d(const MarchArgs &a, int direct, int ind, int prec, int blocks,
                           size_t lds, hipStream_t st) {
  if (direct == PFN_DIRECT_LIGHT_VOLUME)
    return launch_i<VT, PFN_DIRECT_LIGHT_VOLUME>(a, ind, prec, blocks, lds, st);
  return launch_i<VT, PFN_DIRECT_SHADOW_RAYS>(a, ind, prec, blocks, lds, st);
}

hipError_t launch_march(const MarchArgs &a, pfn_dtype vol_dtype, int direct, int ind, int prec,
                        hipStream_t st) {
  size_t lds = 0;
  if (ind == PFN_INDIRECT_FIELD) lds = (size_t)a.mlp_bytes;
  int blocks = ((a.total_blocks + 7) / 8) * 8;
  if (a.persistent) {
    hipLaunchKernelGGL(reset_queues_kernel, dim3(1), dim3(64), 0, st, a.queues);
    int want = 256 * a.persistent;  // workgroups per CU x CUs
    blocks = std::min(blocks, ((want + 7) / 8) * 8);
  }
  if (vol_dtype == PFN_F16) return launch_d<__half>(a, direct, ind, prec, blocks, lds, st);
  return launch_d<float>(a, direct, ind, prec, blocks, lds, st);
}
