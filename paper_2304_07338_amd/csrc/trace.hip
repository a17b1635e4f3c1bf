// Multi-phase photon tracing (Algorithm 1) and the isotropic per-bin photon cache.
//
// One lane per photon path.  Photon `id` belongs to light id mod |L| and HG bin (id/|L|) mod |G|
// (photons split evenly over lights and phases, Section 4.4), leaves the point light in a
// direction drawn uniformly from the cone that contains the cube (the isotropic emission with
// the certain misses removed) with power 4*pi*I*share / N(light, bin), and flies by delta
// tracking with the global majorant.  At every real collision after the first it writes a record (position, incident
// direction, incident power, bin) into its own fixed slots, so records come out in photon order
// without any cross-lane coordination; the throughput is multiplied by the albedo, the direction
// is resampled from HG(g_bin), and Russian roulette may end the path.  Power tallies are kept in
// FP64 per lane, reduced per block and added atomically once per block.
//
// The cache is the collision estimator of the fluence: each record adds Phi / sigma_t(x) with
// cloud-in-cell weights to the 8 nearest cell centres of its bin's grid, scaled by
// 1 / (4 pi V_cell), so a cell holds the direction average of the in-scattered indirect radiance.
#include "pfn_ctx.h"
#include "trace.h"

#define TRACE_THREADS 256
#define N_TALLY 26  // 8 RGB tallies + collisions + null events

template <typename VT>
__global__ __launch_bounds__(TRACE_THREADS) void trace_kernel(TraceArgs a) {
  __shared__ float4 tf[256];
  __shared__ double red[TRACE_THREADS / 64][N_TALLY];
  for (int i = threadIdx.x; i < 256; i += blockDim.x) tf[i] = a.tf[i];
  __syncthreads();

  double tal[N_TALLY];
#pragma unroll
  for (int i = 0; i < N_TALLY; ++i) tal[i] = 0.0;
  const uint64_t groups = (uint64_t)a.n_lights * (uint64_t)a.n_bins;
  const int maxrec = a.max_collisions - 1;
  const VT *vol = reinterpret_cast<const VT *>(a.vol);

  for (uint64_t id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; id < a.n_photons;
       id += (uint64_t)gridDim.x * blockDim.x) {
    const int l = (int)(id % (uint64_t)a.n_lights);
    const int b = (int)((id / (uint64_t)a.n_lights) % (uint64_t)a.n_bins);
    const uint64_t r = (uint64_t)l + (uint64_t)a.n_lights * (uint64_t)b;
    const uint64_t n_lb = a.n_photons / groups + (r < a.n_photons % groups ? 1 : 0);
    const float g = a.g_bins[b];
    Philox rng;
    rng.init(a.seed, id, STREAM_TRACE);
    float ua = rng.next(), ub = rng.next();
    f3 o = {a.light_pos[l][0], a.light_pos[l][1], a.light_pos[l][2]};
    f3 dir;
    float frac = emit_dir(o, ua, ub, dir);
    const float s0 = (float)(4.0 * 3.14159265358979323846 / (double)n_lb) * frac;
    f3 phi0 = {a.light_int[l][0] * s0, a.light_int[l][1] * s0, a.light_int[l][2] * s0};
    tal[0] += phi0.x;  // emitted
    tal[1] += phi0.y;
    tal[2] += phi0.z;
    float t, tmax;
    int nrec = 0;
    if (!clip_cube(o, dir, t, tmax)) {
      tal[6] += phi0.x;  // escaped
      tal[7] += phi0.y;
      tal[8] += phi0.z;
      tal[9] += phi0.x;  // escaped uncollided
      tal[10] += phi0.y;
      tal[11] += phi0.z;
    } else {
      tal[3] += phi0.x;  // entered
      tal[4] += phi0.y;
      tal[5] += phi0.z;
      f3 beta = {1.f, 1.f, 1.f};
      int coll = 0;
      for (;;) {
        if (a.majorant > 0.0f) t += -logf(rng.next()) / a.majorant;
        else t = tmax;
        if (t >= tmax) {
          f3 pw = mul(beta, phi0);
          tal[6] += pw.x;
          tal[7] += pw.y;
          tal[8] += pw.z;
          if (coll == 0) {
            tal[9] += pw.x;
            tal[10] += pw.y;
            tal[11] += pw.z;
          }
          break;
        }
        f3 x = o + dir * t;
        float4 op = tf_lookup(tf, density_at(vol, a.vg, x));
        float sig = op.w * a.ext_scale;
        if (!(rng.next() < sig / a.majorant)) {
          tal[25] += 1.0;
          continue;
        }
        ++coll;
        tal[24] += 1.0;
        f3 pw = mul(beta, phi0);
        if (coll >= 2) {
          uint64_t slot = id * (uint64_t)maxrec + (uint64_t)nrec;
          a.rec_x[3 * slot] = x.x;
          a.rec_x[3 * slot + 1] = x.y;
          a.rec_x[3 * slot + 2] = x.z;
          a.rec_w[3 * slot] = dir.x;
          a.rec_w[3 * slot + 1] = dir.y;
          a.rec_w[3 * slot + 2] = dir.z;
          a.rec_p[3 * slot] = pw.x;
          a.rec_p[3 * slot + 1] = pw.y;
          a.rec_p[3 * slot + 2] = pw.z;
          a.rec_bin[slot] = b;
          ++nrec;
          tal[21] += pw.x;  // stored
          tal[22] += pw.y;
          tal[23] += pw.z;
        }
        f3 alb = {op.x, op.y, op.z};
        tal[12] += (double)pw.x * (1.0 - alb.x);  // absorbed
        tal[13] += (double)pw.y * (1.0 - alb.y);
        tal[14] += (double)pw.z * (1.0 - alb.z);
        beta = mul(beta, alb);
        if (coll >= a.max_collisions) {
          f3 tw = mul(beta, phi0);
          tal[15] += tw.x;  // truncated
          tal[16] += tw.y;
          tal[17] += tw.z;
          break;
        }
        float u1 = rng.next(), u2 = rng.next();
        dir = hg_sample_dir(g, dir, u1, u2);
        if (a.rr_start > 0 && coll >= a.rr_start) {
          float q = fminf(1.0f, maxc(beta));
          if (!(rng.next() < q)) {
            f3 kw = mul(beta, phi0);
            tal[18] += kw.x;  // Russian roulette
            tal[19] += kw.y;
            tal[20] += kw.z;
            break;
          }
          beta = beta * (1.0f / q);
        }
        o = x;
        t = 0.0f;
        tmax = exit_distance(o, dir);
      }
    }
    a.rec_count[id] = (uint8_t)nrec;
  }

  // block reduction of the tallies, then one FP64 atomic per tally per block
  const int lane = lane_id(), wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < N_TALLY; ++i) {
    double v = tal[i];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
    if (lane == 0) red[wave][i] = v;
  }
  __syncthreads();
  if (threadIdx.x < N_TALLY) {
    double v = 0.0;
    for (int w = 0; w < TRACE_THREADS / 64; ++w) v += red[w][threadIdx.x];
    atomicAdd(&a.tally[threadIdx.x], v);
  }
}

// ------------------------------------------------------------------ cache splat
template <typename VT>
__global__ void splat_kernel(SplatArgs a) {
  __shared__ float4 tf[256];
  for (int i = threadIdx.x; i < 256; i += blockDim.x) tf[i] = a.tf[i];
  __syncthreads();
  const int maxrec = a.max_collisions - 1;
  const VT *vol = reinterpret_cast<const VT *>(a.vol);
  const int R = a.res;
  const size_t cells = (size_t)R * R * R;
  const float norm = (float)((double)cells / (4.0 * 3.14159265358979323846));
  for (uint64_t slot = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
       slot < a.n_photons * (uint64_t)maxrec; slot += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t id = slot / (uint64_t)maxrec;
    int k = (int)(slot - id * (uint64_t)maxrec);
    if (k >= (int)a.rec_count[id]) continue;
    f3 x = {a.rec_x[3 * slot], a.rec_x[3 * slot + 1], a.rec_x[3 * slot + 2]};
    float sig = tf_lookup(tf, density_at(vol, a.vg, x)).w * a.ext_scale;
    if (!(sig > 0.0f)) continue;
    float s = norm / sig;
    f3 p = {a.rec_p[3 * slot] * s, a.rec_p[3 * slot + 1] * s, a.rec_p[3 * slot + 2] * s};
    x = clamp01(x);
    int i0, i1, j0, j1, k0, k1;
    float fx, fy, fz;
    tri_axis(x.x, R, i0, i1, fx);
    tri_axis(x.y, R, j0, j1, fy);
    tri_axis(x.z, R, k0, k1, fz);
    float *base = reinterpret_cast<float *>(a.cache + (size_t)a.rec_bin[slot] * cells);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      int ix = (c & 1) ? i1 : i0, iy = (c & 2) ? j1 : j0, iz = (c & 4) ? k1 : k0;
      float w = ((c & 1) ? fx : 1.0f - fx) * ((c & 2) ? fy : 1.0f - fy) * ((c & 4) ? fz : 1.0f - fz);
      float *e = base + (((size_t)iz * R + iy) * R + ix) * 4;
      atomicAdd(e + 0, w * p.x);
      atomicAdd(e + 1, w * p.y);
      atomicAdd(e + 2, w * p.z);
    }
  }
}

// Maximum of the cache (non-negative floats order like their bit patterns).
__global__ void cache_max_kernel(const float4 *__restrict__ c, size_t cells, unsigned *out) {
  float m = 0.0f;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < cells;
       i += (size_t)gridDim.x * blockDim.x) {
    float4 v = c[i];
    m = fmaxf(m, fmaxf(v.x, fmaxf(v.y, v.z)));
  }
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_down(m, off));
  if (lane_id() == 0) atomicMax(out, __float_as_uint(m));
}

__global__ void cache_pack_kernel(const float *__restrict__ src, float4 *__restrict__ dst,
                                  size_t cells) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cells) dst[i] = make_float4(src[3 * i], src[3 * i + 1], src[3 * i + 2], 0.0f);
}
__global__ void cache_unpack_kernel(const float4 *__restrict__ src, float *__restrict__ dst,
                                    size_t cells) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cells) {
    float4 v = src[i];
    dst[3 * i] = v.x;
    dst[3 * i + 1] = v.y;
    dst[3 * i + 2] = v.z;
  }
}

hipError_t launch_cache_pack(pfn_context *ctx, const float *src, size_t cells) {
  hipLaunchKernelGGL(cache_pack_kernel, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0,
                     ctx->stream, src, ctx->cache, cells);
  return hipGetLastError();
}
hipError_t launch_cache_unpack(pfn_context *ctx, float *dst, size_t cells) {
  hipLaunchKernelGGL(cache_unpack_kernel, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0,
                     ctx->stream, ctx->cache, dst, cells);
  return hipGetLastError();
}

// Records of the last trace, compacted in photon order.
__global__ void record_offsets_kernel(const uint8_t *__restrict__ cnt, uint64_t n,
                                      unsigned long long *__restrict__ block_sums, int per_block) {
  // per-block sums of record counts (one block covers per_block photons)
  __shared__ unsigned long long red[4];
  uint64_t begin = (uint64_t)blockIdx.x * per_block;
  unsigned long long s = 0;
  for (uint64_t i = begin + threadIdx.x; i < n && i < begin + per_block; i += blockDim.x) s += cnt[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off);
  if (lane_id() == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) block_sums[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void record_copy_kernel(RecordCopyArgs a) {
  // one block per photon chunk; a serial scan inside the block over its photons (256 threads
  // cooperate per photon chunk of per_block photons, thread 0 computes running offsets in LDS)
  __shared__ unsigned long long offs[1024];
  uint64_t begin = (uint64_t)blockIdx.x * a.per_block;
  uint64_t end = begin + a.per_block < a.n ? begin + a.per_block : a.n;
  if (threadIdx.x == 0) {
    unsigned long long o = a.block_offsets[blockIdx.x];
    for (uint64_t i = begin; i < end; ++i) {
      offs[i - begin] = o;
      o += a.cnt[i];
    }
  }
  __syncthreads();
  for (uint64_t i = begin + threadIdx.x; i < end; i += blockDim.x) {
    unsigned long long o = offs[i - begin];
    for (int k = 0; k < a.cnt[i]; ++k) {
      unsigned long long dst = o + k;
      if (dst >= a.capacity) break;
      uint64_t src = i * (uint64_t)a.maxrec + k;
      for (int c = 0; c < 3; ++c) {
        if (a.x) a.x[3 * dst + c] = a.src_x[3 * src + c];
        if (a.w) a.w[3 * dst + c] = a.src_w[3 * src + c];
        if (a.p) a.p[3 * dst + c] = a.src_p[3 * src + c];
      }
      if (a.bin) a.bin[dst] = a.src_bin[src];
      if (a.photon) a.photon[dst] = (int64_t)i;
    }
  }
}

// ------------------------------------------------------------------ host API
static pfn_status trace_alloc(pfn_context *ctx, uint64_t slots, uint64_t photons) {
  if (ctx->rec_cap >= slots && ctx->cnt_cap >= photons) return PFN_OK;
  auto fr = [](void *p) {
    if (p) (void)hipFree(p);
  };
  fr(ctx->rec_x);
  fr(ctx->rec_w);
  fr(ctx->rec_p);
  fr(ctx->rec_bin);
  fr(ctx->rec_cnt);
  ctx->rec_x = ctx->rec_w = ctx->rec_p = nullptr;
  ctx->rec_bin = nullptr;
  ctx->rec_cnt = nullptr;
  ctx->rec_cap = ctx->cnt_cap = 0;
  ctx->rec_photons = ctx->rec_count = 0;  // the old records are gone, also if allocation fails
  PFN_HIP(ctx, hipMalloc((void **)&ctx->rec_x, slots * 12));
  PFN_HIP(ctx, hipMalloc((void **)&ctx->rec_w, slots * 12));
  PFN_HIP(ctx, hipMalloc((void **)&ctx->rec_p, slots * 12));
  PFN_HIP(ctx, hipMalloc((void **)&ctx->rec_bin, slots * 4));
  PFN_HIP(ctx, hipMalloc((void **)&ctx->rec_cnt, photons));
  ctx->rec_cap = slots;
  ctx->cnt_cap = photons;
  return PFN_OK;
}

extern "C" pfn_status pfn_trace_photon_cache(pfn_context *ctx, const pfn_trace_params *p,
                                             pfn_trace_stats *stats) {
  if (!ctx) return PFN_ERR_INVALID_ARG;
  if (!p) return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "params are NULL");
  if (p->n_photons < 1 || p->n_photons > (1ull << 34))
    return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "n_photons in [1, 2^34]");
  if (p->n_bins < 1 || p->n_bins > 8) return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "1 to 8 bins");
  for (int b = 0; b < p->n_bins; ++b) {
    if (!(std::fabs(p->g_bins[b]) <= 0.95f))
      return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "|g| <= 0.95");
    if (b && !(p->g_bins[b] > p->g_bins[b - 1]))
      return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "g bins must be ascending");
  }
  if (p->cache_res < 2 || p->cache_res > 512)
    return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "cache_res in [2, 512]");
  if (p->max_collisions < 1 || p->max_collisions > 64)
    return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "max_collisions in [1, 64]");
  if (!ctx->vol || !ctx->tf_set || ctx->n_lights < 1)
    return pfn_fail(ctx, PFN_ERR_NOT_READY, "trace needs volume, transfer function and lights");
  PFN_HIP(ctx, hipSetDevice(ctx->device));
  const int maxrec = p->max_collisions > 1 ? p->max_collisions - 1 : 1;
  uint64_t slots = p->n_photons * (uint64_t)maxrec;
  pfn_status st = trace_alloc(ctx, slots, p->n_photons);
  if (st) return st;
  st = ensure_scratch(ctx, 64 * sizeof(double));
  if (st) return st;
  double *tally = (double *)ctx->scratch;
  PFN_HIP(ctx, hipMemsetAsync(tally, 0, 64 * sizeof(double), ctx->stream));

  TraceArgs a{};
  a.vol = ctx->vol;
  a.vg = ctx->vol_grid;
  a.tf = ctx->tf_dev;
  a.ext_scale = ctx->ext_scale;
  a.majorant = ctx->majorant;
  a.n_lights = ctx->n_lights;
  for (int l = 0; l < ctx->n_lights; ++l)
    for (int c = 0; c < 3; ++c) {
      a.light_pos[l][c] = ctx->lights[l].pos[c];
      a.light_int[l][c] = ctx->lights[l].intensity[c];
    }
  a.n_bins = p->n_bins;
  for (int b = 0; b < p->n_bins; ++b) a.g_bins[b] = p->g_bins[b];
  a.max_collisions = p->max_collisions;
  a.rr_start = p->rr_start;
  a.seed = p->seed;
  a.n_photons = p->n_photons;
  a.rec_x = ctx->rec_x;
  a.rec_w = ctx->rec_w;
  a.rec_p = ctx->rec_p;
  a.rec_bin = ctx->rec_bin;
  a.rec_count = ctx->rec_cnt;
  a.tally = tally;
  uint64_t want = (p->n_photons + TRACE_THREADS - 1) / TRACE_THREADS;
  unsigned blocks = (unsigned)(want < 256 * 32 ? want : 256 * 32);
  const int tslot = timing_begin(ctx);
  if (ctx->vol_dtype == PFN_F16)
    hipLaunchKernelGGL(trace_kernel<__half>, dim3(blocks), dim3(TRACE_THREADS), 0, ctx->stream, a);
  else
    hipLaunchKernelGGL(trace_kernel<float>, dim3(blocks), dim3(TRACE_THREADS), 0, ctx->stream, a);
  PFN_HIP(ctx, hipGetLastError());
  timing_end(ctx, tslot, TK_TRACE);
  ctx->rec_photons = p->n_photons;
  ctx->rec_maxrec = maxrec;

  // cache
  st = alloc_cache(ctx, p->n_bins, p->cache_res);
  if (st) return st;
  size_t cells = (size_t)p->cache_res * p->cache_res * p->cache_res;
  PFN_HIP(ctx, hipMemsetAsync(ctx->cache, 0, cells * p->n_bins * sizeof(float4), ctx->stream));
  SplatArgs s{};
  s.vol = ctx->vol;
  s.vg = ctx->vol_grid;
  s.tf = ctx->tf_dev;
  s.ext_scale = ctx->ext_scale;
  s.res = p->cache_res;
  s.max_collisions = p->max_collisions > 1 ? p->max_collisions : 2;
  s.n_photons = p->n_photons;
  s.rec_x = ctx->rec_x;
  s.rec_p = ctx->rec_p;
  s.rec_bin = ctx->rec_bin;
  s.rec_count = ctx->rec_cnt;
  s.cache = ctx->cache;
  uint64_t sw = (slots + 255) / 256;
  unsigned sblocks = (unsigned)(sw < 256 * 64 ? sw : 256 * 64);
  if (ctx->vol_dtype == PFN_F16)
    hipLaunchKernelGGL(splat_kernel<__half>, dim3(sblocks), dim3(256), 0, ctx->stream, s);
  else
    hipLaunchKernelGGL(splat_kernel<float>, dim3(sblocks), dim3(256), 0, ctx->stream, s);
  PFN_HIP(ctx, hipGetLastError());
  unsigned *kmax = (unsigned *)(tally + 32);
  size_t tot = cells * p->n_bins;
  unsigned mblocks = (unsigned)std::min<size_t>((tot + 255) / 256, 4096);
  hipLaunchKernelGGL(cache_max_kernel, dim3(mblocks), dim3(256), 0, ctx->stream, ctx->cache, tot,
                     kmax);
  PFN_HIP(ctx, hipGetLastError());

  double host[33];
  PFN_HIP(ctx, hipMemcpyAsync(host, tally, sizeof(host), hipMemcpyDeviceToHost, ctx->stream));
  // record total
  uint8_t dummy = 0;
  (void)dummy;
  PFN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  unsigned kbits;
  std::memcpy(&kbits, &host[32], sizeof(unsigned));
  float kf;
  std::memcpy(&kf, &kbits, sizeof(float));
  for (int b = 0; b < p->n_bins; ++b) ctx->g_bins[b] = p->g_bins[b];
  ctx->kappa = kf > 0.0f ? (double)kf : 1.0;
  ctx->cache_valid = true;

  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    double *dst = &stats->emitted[0];
    for (int i = 0; i < N_TALLY; ++i) dst[i] = host[i];
    stats->kappa = ctx->kappa;
  }
  // count records (sum of per-photon counts)
  uint64_t nrec = 0;
  st = count_records(ctx, &nrec);
  if (st) return st;
  ctx->rec_count = nrec;
  if (stats) {
    stats->n_records = nrec;
    stats->n_records_dropped = 0;
  }
  return PFN_OK;
}

pfn_status count_records(pfn_context *ctx, uint64_t *out) {
  const uint64_t n = ctx->rec_photons;
  const int per_block = 1024;
  uint64_t nb = (n + per_block - 1) / per_block;
  pfn_status st = ensure_scratch(ctx, 64 * sizeof(double) + (nb + 1) * 8);
  if (st) return st;
  unsigned long long *sums = (unsigned long long *)((char *)ctx->scratch + 64 * sizeof(double));
  hipLaunchKernelGGL(record_offsets_kernel, dim3((unsigned)nb), dim3(256), 0, ctx->stream,
                     ctx->rec_cnt, n, sums, per_block);
  PFN_HIP(ctx, hipGetLastError());
  std::vector<unsigned long long> h(nb);
  PFN_HIP(ctx, hipMemcpyAsync(h.data(), sums, nb * 8, hipMemcpyDeviceToHost, ctx->stream));
  PFN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  uint64_t tot = 0;
  for (auto v : h) tot += v;
  *out = tot;
  return PFN_OK;
}

extern "C" pfn_status pfn_get_records(pfn_context *ctx, float *x, float *w, float *pw,
                                      int32_t *bin, int64_t *photon, uint64_t capacity,
                                      uint64_t *count) {
  if (!ctx) return PFN_ERR_INVALID_ARG;
  if (!count) return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "count is NULL");
  if (ctx->rec_photons == 0) return pfn_fail(ctx, PFN_ERR_NOT_READY, "no trace yet");
  PFN_HIP(ctx, hipSetDevice(ctx->device));
  const uint64_t n = ctx->rec_photons;
  const int per_block = 1024;
  uint64_t nb = (n + per_block - 1) / per_block;
  pfn_status st = ensure_scratch(ctx, 64 * sizeof(double) + (nb + 1) * 8);
  if (st) return st;
  unsigned long long *sums = (unsigned long long *)((char *)ctx->scratch + 64 * sizeof(double));
  hipLaunchKernelGGL(record_offsets_kernel, dim3((unsigned)nb), dim3(256), 0, ctx->stream,
                     ctx->rec_cnt, n, sums, per_block);
  PFN_HIP(ctx, hipGetLastError());
  std::vector<unsigned long long> h(nb);
  PFN_HIP(ctx, hipMemcpyAsync(h.data(), sums, nb * 8, hipMemcpyDeviceToHost, ctx->stream));
  PFN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  unsigned long long acc = 0;
  for (auto &v : h) {
    unsigned long long t = v;
    v = acc;
    acc += t;
  }
  PFN_HIP(ctx, hipMemcpyAsync(sums, h.data(), nb * 8, hipMemcpyHostToDevice, ctx->stream));
  RecordCopyArgs a{};
  a.cnt = ctx->rec_cnt;
  a.n = n;
  a.per_block = per_block;
  a.block_offsets = sums;
  a.capacity = capacity;
  a.maxrec = ctx->rec_maxrec;
  a.src_x = ctx->rec_x;
  a.src_w = ctx->rec_w;
  a.src_p = ctx->rec_p;
  a.src_bin = ctx->rec_bin;
  a.x = x;
  a.w = w;
  a.p = pw;
  a.bin = bin;
  a.photon = photon;
  hipLaunchKernelGGL(record_copy_kernel, dim3((unsigned)nb), dim3(256), 0, ctx->stream, a);
  PFN_HIP(ctx, hipGetLastError());
  PFN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  *count = acc < capacity ? acc : capacity;
  return PFN_OK;
}
