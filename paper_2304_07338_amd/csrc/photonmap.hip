// Photon map and the radiance estimate of Eq. (5) (Section 3.3).
//
// Build: the photon records (of the last trace, or given by the caller) get a key (HG bin, cell
// of a uniform G^3 grid) and are counting-sorted by it: one pass counts the keys with atomics,
// an exclusive scan gives every key's first record, a second pass scatters the records.  Each
// sorted record holds its position, incident direction and the collision-estimator score
// Phi / sigma_t(x) (RGB), 36 bytes.  Records of one cell end up in an arbitrary order, so sums
// over them are reproducible only up to FP32 rounding.
//
// Estimate: one wave per query.  The cells that the query's sphere of radius R touches form a
// box; along x the cells of one (bin, z, y) row are one contiguous run of records, so the wave
// streams runs, 64 records at a time.
//   - fixed radius (k = 0): every record of the query's bin within R, divided by (4/3) pi R^3;
//   - K nearest (k > 0): the records within R are histogrammed in LDS by (d/R)^3 (1024 bins);
//     the bin where the running count reaches k is refined by further histograms until it holds
//     at most 256 records, which are then ranked by distance in LDS.  The k nearest are summed
//     and divided by the sphere through the farthest of them (all records within R, and the
//     farthest of those, if there are at most k).
// A record's contribution is p_g(w_n . w) * score, with g the bin's anisotropy.
#include "pfn_ctx.h"

#define PM_THREADS 256
#define PM_NB 1024          // histogram bins per refinement level
#define PM_CAP 256          // records ranked in LDS
#define PM_LEVELS 4         // refinement levels

struct PmSrc {
  const float *x, *w, *p;
  const int32_t *bin;
  const uint8_t *cnt;  // records per photon (slotted trace records), or NULL: every slot valid
  int maxrec;
  uint64_t n_slots;
  uint64_t i0;         // first slot of this launch (a build over more slots than one dispatch
                       // holds runs in pieces)
};

__device__ __forceinline__ bool pm_valid(const PmSrc &s, uint64_t i) {
  if (!s.cnt) return true;
  const uint64_t ph = i / (uint64_t)s.maxrec;
  return (int)(i - ph * (uint64_t)s.maxrec) < (int)s.cnt[ph];
}

__device__ __forceinline__ int pm_cell(float v, int G) {
  int c = (int)floorf(v * (float)G);
  return c < 0 ? 0 : (c >= G ? G - 1 : c);
}

__global__ void pm_count_kernel(PmSrc s, int G, int n_bins, uint32_t *__restrict__ counts,
                                uint32_t *__restrict__ keys) {
  const uint64_t i = s.i0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.n_slots) return;
  uint32_t key = 0xFFFFFFFFu;
  if (pm_valid(s, i)) {
    const int b = s.bin[i];
    if (b >= 0 && b < n_bins) {
      const int cx = pm_cell(s.x[3 * i], G), cy = pm_cell(s.x[3 * i + 1], G),
                cz = pm_cell(s.x[3 * i + 2], G);
      key = (uint32_t)((((int64_t)b * G + cz) * G + cy) * G + cx);
      atomicAdd(&counts[key], 1u);
    }
  }
  keys[i] = key;
}

// Exclusive scan of 1024-element blocks; block totals go to `sums`.
__global__ __launch_bounds__(256) void pm_scan_block_kernel(const uint32_t *__restrict__ in,
                                                            uint32_t *__restrict__ out,
                                                            uint32_t *__restrict__ sums,
                                                            uint64_t n) {
  __shared__ uint32_t wsum[4];
  const uint64_t base = (uint64_t)blockIdx.x * 1024 + (uint64_t)threadIdx.x * 4;
  uint32_t v[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) v[j] = base + j < n ? in[base + j] : 0u;
  const uint32_t t = v[0] + v[1] + v[2] + v[3];
  // inclusive scan of the thread totals within the wave, then across the 4 waves
  uint32_t inc = t;
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == 63) wsum[threadIdx.x >> 6] = inc;
  __syncthreads();
  uint32_t wbase = 0;
  for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) wbase += wsum[w];
  uint32_t run = wbase + inc - t;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (base + j < n) out[base + j] = run;
    run += v[j];
  }
  if (threadIdx.x == 255 && sums) sums[blockIdx.x] = wbase + inc;
}

__global__ void pm_add_kernel(uint32_t *__restrict__ out, const uint32_t *__restrict__ offs,
                              uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += offs[i >> 10];
}

struct PmScatterArgs {
  PmSrc s;
  const uint32_t *keys, *start;
  uint32_t *fill;
  const void *vol;
  BrickGrid vg;
  const float4 *tf;
  float ext_scale;
  float4 *ra, *rb;
  float *rc;
};

template <typename VT>
__global__ void pm_scatter_kernel(PmScatterArgs a) {
  const uint64_t i = a.s.i0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.s.n_slots) return;
  const uint32_t key = a.keys[i];
  if (key == 0xFFFFFFFFu) return;
  const uint32_t dst = a.start[key] + atomicAdd(&a.fill[key], 1u);
  const f3 x = {a.s.x[3 * i], a.s.x[3 * i + 1], a.s.x[3 * i + 2]};
  const float sig =
      tf_lookup(a.tf, density_at(reinterpret_cast<const VT *>(a.vol), a.vg, x)).w * a.ext_scale;
  const float inv = sig > 0.0f ? 1.0f / sig : 0.0f;
  a.ra[dst] = make_float4(x.x, x.y, x.z, a.s.p[3 * i] * inv);
  a.rb[dst] = make_float4(a.s.w[3 * i], a.s.w[3 * i + 1], a.s.w[3 * i + 2], a.s.p[3 * i + 1] * inv);
  a.rc[dst] = a.s.p[3 * i + 2] * inv;
}

// ------------------------------------------------------------------ estimate
struct PmEstArgs {
  const float4 *ra, *rb;
  const float *rc;
  const uint32_t *start;
  int G, n_bins;
  float g_bins[8];
  const float *qx, *qw;
  const int32_t *qbin;
  int64_t q0, n;        // queries q0 .. n-1 (one wave each; larger batches run in pieces)
  float radius;
  int k;
  float *out, *r_out;
  int32_t *n_out;
};

struct PmWaveLds {
  uint32_t hist[PM_NB];
  float d2[PM_CAP];
  float c[PM_CAP][3];
  uint32_t n_buf;
};

// Distance from v to the cell interval [c / G, (c + 1) / G] along one axis (0 inside).
__device__ __forceinline__ float pm_gap(float v, int c, float inv_g) {
  const float lo = (float)c * inv_g, hi = (float)(c + 1) * inv_g;
  return fmaxf(fmaxf(lo - v, v - hi), 0.0f);
}

// Visits the records of bin b in the cells that the sphere of radius R around x touches:
// f(d2, record) per record, the wave's lanes taking 64 consecutive records at a time.  A
// (z, y) row of cells is skipped when its nearest point is farther than R, and within a row
// only the cells under the sphere's chord are read.  Both tests use R (1 + 1e-5) + 1e-6, a
// margin above the FP32 rounding of cell bounds and coordinates (a few 1e-7), so that no record
// that the FP32 test d2 <= R^2 accepts is missed.
template <typename F>
__device__ __forceinline__ void pm_for_candidates(const PmEstArgs &a, int b, f3 x, F &&f) {
  const int G = a.G;
  const float R = a.radius, Rm = R * (1.0f + 1e-5f) + 1e-6f, R2m = Rm * Rm;
  const float inv_g = 1.0f / (float)G;
  const int y0 = pm_cell(x.y - Rm, G), y1 = pm_cell(x.y + Rm, G);
  const int z0 = pm_cell(x.z - Rm, G), z1 = pm_cell(x.z + Rm, G);
  const uint32_t lane = (uint32_t)lane_id();
  for (int cz = z0; cz <= z1; ++cz) {
    const float gz = pm_gap(x.z, cz, inv_g);
    for (int cy = y0; cy <= y1; ++cy) {
      const float gy = pm_gap(x.y, cy, inv_g);
      const float rest = R2m - gz * gz - gy * gy;
      if (rest < 0.0f) continue;
      const float half = sqrtf(rest) * (1.0f + 1e-5f) + 1e-6f;
      const int x0 = pm_cell(x.x - half, G), x1 = pm_cell(x.x + half, G);
      const int64_t row = (((int64_t)b * G + cz) * G + cy) * G;
      const uint32_t s0 = a.start[row + x0], s1 = a.start[row + x1 + 1];
      // two records per lane per pass: both loads are in flight together
      for (uint32_t j = s0 + lane; j < s1; j += 128) {
        const uint32_t j2 = j + 64;
        const bool two = j2 < s1;
        const float4 p = a.ra[j];
        const float4 p2 = two ? a.ra[j2] : p;
        float dx = p.x - x.x, dy = p.y - x.y, dz = p.z - x.z;
        f(dx * dx + dy * dy + dz * dz, j);
        if (two) {
          dx = p2.x - x.x;
          dy = p2.y - x.y;
          dz = p2.z - x.z;
          f(dx * dx + dy * dy + dz * dz, j2);
        }
      }
    }
  }
}

__device__ __forceinline__ float pm_wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ uint32_t pm_wave_sum_u(uint32_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ float pm_wave_max(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

// Histogram bin of u in the level range [lo, lo + wd).
__device__ __forceinline__ int pm_idx(float u, float lo, float wd) {
  const int h = (int)((u - lo) / wd * (float)PM_NB);
  return h < 0 ? 0 : (h >= PM_NB ? PM_NB - 1 : h);
}

// The bin where the running count of the wave's LDS histogram reaches `need`: returns it and
// the count before it.
__device__ __forceinline__ int pm_crossing(const PmWaveLds &L, uint32_t need, uint32_t &before) {
  const int lane = lane_id();
  constexpr int PER = PM_NB / 64;
  uint32_t own = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) own += L.hist[lane * PER + j];
  uint32_t inc = own;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  const uint64_t m = __builtin_amdgcn_ballot_w64(inc >= need);
  const int src = m ? __builtin_ctzll(m) : 63;
  uint32_t run = __shfl(inc - own, src);
  int bin = src * PER + PER - 1;
  for (int j = 0; j < PER; ++j) {
    const uint32_t h = L.hist[src * PER + j];
    if (run + h >= need) {
      bin = src * PER + j;
      break;
    }
    run += h;
  }
  before = run;
  return bin;
}

template <bool KNN>
__global__ __launch_bounds__(64) void pm_estimate_kernel(PmEstArgs a) {
  __shared__ PmWaveLds L;
  const int64_t q = a.q0 + blockIdx.x;
  if (q >= a.n) return;
  const int lane = lane_id();
  const f3 x = {a.qx[3 * q], a.qx[3 * q + 1], a.qx[3 * q + 2]};
  const f3 w = {a.qw[3 * q], a.qw[3 * q + 1], a.qw[3 * q + 2]};
  const int b = a.qbin[q];
  auto store = [&](f3 v, float r, int n) {
    if (lane == 0) {
      a.out[3 * q] = v.x;
      a.out[3 * q + 1] = v.y;
      a.out[3 * q + 2] = v.z;
      if (a.r_out) a.r_out[q] = r;
      if (a.n_out) a.n_out[q] = n;
    }
  };
  if (b < 0 || b >= a.n_bins) {
    store(f3{0.f, 0.f, 0.f}, 0.0f, 0);
    return;
  }
  const float g = a.g_bins[b];
  const float hg_c = (1.0f - g * g) * (0.25f / PFN_PI), hg_a = 1.0f + g * g, hg_b = 2.0f * g;
  // p_g(w_n . w) * score of record j
  auto contrib = [&](uint32_t j) {
    const float4 p = a.ra[j], d = a.rb[j];
    const float sb = a.rc[j];
    const float mu = d.x * w.x + d.y * w.y + d.z * w.z;
    const float rd = rsqrtf(fmaf(-hg_b, mu, hg_a));
    const float ph = hg_c * (rd * rd * rd);
    return f3{ph * p.w, ph * d.w, ph * sb};
  };
  const float R = a.radius, R2 = R * R;
  const float k43pi = 4.0f / 3.0f * PFN_PI;

  if constexpr (!KNN) {
    f3 S = {0.f, 0.f, 0.f};
    uint32_t cnt = 0;
    pm_for_candidates(a, b, x, [&](float d2, uint32_t j) {
      if (d2 <= R2) {
        S = S + contrib(j);
        ++cnt;
      }
    });
    const float inv = 1.0f / (k43pi * R2 * R);
    const uint32_t n = pm_wave_sum_u(cnt);
    store(f3{pm_wave_sum(S.x) * inv, pm_wave_sum(S.y) * inv, pm_wave_sum(S.z) * inv}, R, (int)n);
    return;
  } else {
    const uint32_t k = (uint32_t)a.k;
    auto u_of = [&](float d2) {
      const float t = d2 / R2;
      return t * sqrtf(t);  // (d / R)^3: equal-volume shells
    };
    // pass 1: count, sums and the farthest distance of every record within R; histogram
    for (int i = lane; i < PM_NB; i += 64) L.hist[i] = 0u;
    __syncthreads();
    f3 S = {0.f, 0.f, 0.f};
    uint32_t cnt = 0;
    float dmax = 0.0f;
    pm_for_candidates(a, b, x, [&](float d2, uint32_t j) {
      if (d2 <= R2) {
        S = S + contrib(j);
        ++cnt;
        dmax = fmaxf(dmax, d2);
        atomicAdd(&L.hist[pm_idx(u_of(d2), 0.0f, 1.0f)], 1u);
      }
    });
    __syncthreads();
    const uint32_t total = pm_wave_sum_u(cnt);
    if (total <= k) {
      const float r2 = pm_wave_max(dmax);
      const float r = sqrtf(r2);
      const float inv = total > 0 && r > 0.0f ? 1.0f / (k43pi * r2 * r) : 0.0f;
      store(f3{pm_wave_sum(S.x) * inv, pm_wave_sum(S.y) * inv, pm_wave_sum(S.z) * inv},
            total > 0 ? r : 0.0f, (int)total);
      return;
    }
    // the bin holding the k-th nearest, refined until it holds at most PM_CAP records
    float lo[PM_LEVELS], wd[PM_LEVELS];
    int bs[PM_LEVELS];
    int nlev = 0;
    uint32_t need = k;
    float l0 = 0.0f, w0 = 1.0f;
    auto classify = [&](float u) {
      for (int l = 0; l < nlev; ++l) {
        const int h = pm_idx(u, lo[l], wd[l]);
        if (h != bs[l]) return h < bs[l] ? -1 : 1;
      }
      return 0;
    };
    for (;;) {
      uint32_t before = 0;
      const int bstar = pm_crossing(L, need, before);
      const uint32_t in_bin = L.hist[bstar];
      lo[nlev] = l0;
      wd[nlev] = w0;
      bs[nlev] = bstar;
      ++nlev;
      need -= before;
      if (in_bin <= PM_CAP || nlev == PM_LEVELS) break;
      l0 = l0 + (float)bstar * w0 / (float)PM_NB;
      w0 = w0 / (float)PM_NB;
      __syncthreads();
      for (int i = lane; i < PM_NB; i += 64) L.hist[i] = 0u;
      __syncthreads();
      pm_for_candidates(a, b, x, [&](float d2, uint32_t j) {
        if (d2 <= R2) {
          const float u = u_of(d2);
          if (classify(u) == 0) atomicAdd(&L.hist[pm_idx(u, l0, w0)], 1u);
        }
      });
      __syncthreads();
    }
    // collect pass: records below the final bin are summed, those in it ranked in LDS
    if (lane == 0) L.n_buf = 0u;
    __syncthreads();
    f3 A = {0.f, 0.f, 0.f};
    pm_for_candidates(a, b, x, [&](float d2, uint32_t j) {
      if (d2 <= R2) {
        const int c = classify(u_of(d2));
        if (c < 0) {
          A = A + contrib(j);
        } else if (c == 0) {
          const uint32_t slot = atomicAdd(&L.n_buf, 1u);
          if (slot < PM_CAP) {
            const f3 v = contrib(j);
            L.d2[slot] = d2;
            L.c[slot][0] = v.x;
            L.c[slot][1] = v.y;
            L.c[slot][2] = v.z;
          }
        }
      }
    });
    __syncthreads();
    const int nbuf = (int)min(L.n_buf, (uint32_t)PM_CAP);
    float rfar = 0.0f;
    for (int e = lane; e < nbuf; e += 64) {
      const float de = L.d2[e];
      uint32_t rank = 0;
      for (int f = 0; f < nbuf; ++f) {
        const float df = L.d2[f];
        rank += (df < de || (df == de && f < e)) ? 1u : 0u;
      }
      if (rank < need) {
        A = A + f3{L.c[e][0], L.c[e][1], L.c[e][2]};
        rfar = fmaxf(rfar, de);
      }
    }
    const float r2 = pm_wave_max(rfar);
    const float r = sqrtf(r2);
    const float inv = r > 0.0f ? 1.0f / (k43pi * r2 * r) : 0.0f;
    store(f3{pm_wave_sum(A.x) * inv, pm_wave_sum(A.y) * inv, pm_wave_sum(A.z) * inv}, r, (int)k);
  }
}

// ------------------------------------------------------------------ host side
static hipError_t pm_scan(PhotonMapState &m, const uint32_t *in, uint32_t *out, uint64_t n,
                          int depth, hipStream_t st) {
  const uint64_t blocks = (n + 1023) / 1024;
  uint32_t *sums = m.scan_tmp[depth], *sums_scanned = m.scan_tmp[depth] + blocks;
  hipLaunchKernelGGL(pm_scan_block_kernel, dim3((unsigned)blocks), dim3(256), 0, st, in, out,
                     blocks > 1 ? sums : nullptr, n);
  if (blocks > 1) {
    hipError_t e = pm_scan(m, sums, sums_scanned, blocks, depth + 1, st);
    if (e) return e;
    hipLaunchKernelGGL(pm_add_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, out,
                       sums_scanned, n);
  }
  return hipGetLastError();
}

static void pm_free(PhotonMapState &m) {
  auto fr = [](auto *&p) {
    if (p) (void)hipFree((void *)p);
    p = nullptr;
  };
  fr(m.ra);
  fr(m.rb);
  fr(m.rc);
  fr(m.start);
  fr(m.counts);
  fr(m.keys);
  for (auto &t : m.scan_tmp) fr(t);
  m.rec_cap = m.slot_cap = m.key_cap = 0;
  m.valid = false;
}

void pm_release(PhotonMapState &m) { pm_free(m); }

pfn_status pm_build(pfn_context *ctx, const PmSrcHost &src, int n_bins, const float *g_bins,
                    int G) {
  PhotonMapState &m = ctx->pmap;
  m.valid = false;
  const uint64_t n_keys = (uint64_t)n_bins * G * G * G;
  if (n_keys + 1 > m.key_cap) {
    if (m.start) (void)hipFree(m.start);
    if (m.counts) (void)hipFree(m.counts);
    for (auto &t : m.scan_tmp)
      if (t) (void)hipFree(t), t = nullptr;
    m.start = m.counts = nullptr;
    m.key_cap = 0;
    PFN_HIP(ctx, hipMalloc((void **)&m.start, sizeof(uint32_t) * (n_keys + 1)));
    PFN_HIP(ctx, hipMalloc((void **)&m.counts, sizeof(uint32_t) * (n_keys + 1)));
    // block sums of the scan levels: 1024-fold fewer per level
    uint64_t len = n_keys + 1;
    for (int d = 0; d < PM_SCAN_DEPTH; ++d) {
      len = (len + 1023) / 1024;
      PFN_HIP(ctx, hipMalloc((void **)&m.scan_tmp[d], sizeof(uint32_t) * 2 * (len + 1)));
    }
    m.key_cap = n_keys + 1;
  }
  if (src.n_slots > m.slot_cap) {
    if (m.keys) (void)hipFree(m.keys);
    m.keys = nullptr;
    m.slot_cap = 0;
    PFN_HIP(ctx, hipMalloc((void **)&m.keys, sizeof(uint32_t) * src.n_slots));
    m.slot_cap = src.n_slots;
  }
  hipStream_t st = ctx->stream;
  PmSrc s{src.x, src.w, src.p, src.bin, src.cnt, src.maxrec, src.n_slots, 0};
  PFN_HIP(ctx, hipMemsetAsync(m.counts, 0, sizeof(uint32_t) * (n_keys + 1), st));
  // one work-item per slot, in pieces of at most PFN_DISPATCH_ITEMS slots
  const uint64_t piece = (uint64_t)PFN_DISPATCH_ITEMS;
  auto piece_blocks = [&](uint64_t i0) {
    return dim3((unsigned)((std::min(src.n_slots - i0, piece) + 255) / 256));
  };
  for (s.i0 = 0; s.i0 < src.n_slots; s.i0 += piece) {
    hipLaunchKernelGGL(pm_count_kernel, piece_blocks(s.i0), dim3(256), 0, st, s, G, n_bins,
                       m.counts, m.keys);
    PFN_HIP(ctx, hipGetLastError());
  }
  PFN_HIP(ctx, pm_scan(m, m.counts, m.start, n_keys + 1, 0, st));
  uint32_t total = 0;
  PFN_HIP(ctx, hipMemcpyAsync(&total, m.start + n_keys, 4, hipMemcpyDeviceToHost, st));
  PFN_HIP(ctx, hipStreamSynchronize(st));
  if (total > m.rec_cap) {
    auto fr = [](auto *&p) {
      if (p) (void)hipFree((void *)p);
      p = nullptr;
    };
    fr(m.ra);
    fr(m.rb);
    fr(m.rc);
    m.rec_cap = 0;
    PFN_HIP(ctx, hipMalloc((void **)&m.ra, sizeof(float4) * total));
    PFN_HIP(ctx, hipMalloc((void **)&m.rb, sizeof(float4) * total));
    PFN_HIP(ctx, hipMalloc((void **)&m.rc, sizeof(float) * total));
    m.rec_cap = total;
  }
  // the counts become the fill counters of the scatter
  PFN_HIP(ctx, hipMemsetAsync(m.counts, 0, sizeof(uint32_t) * (n_keys + 1), st));
  PmScatterArgs a{};
  a.s = s;
  a.keys = m.keys;
  a.start = m.start;
  a.fill = m.counts;
  a.vol = ctx->vol;
  a.vg = ctx->vol_grid;
  a.tf = ctx->tf_dev;
  a.ext_scale = ctx->ext_scale;
  a.ra = m.ra;
  a.rb = m.rb;
  a.rc = m.rc;
  for (a.s.i0 = 0; a.s.i0 < src.n_slots; a.s.i0 += piece) {
    if (ctx->vol_dtype == PFN_F16)
      hipLaunchKernelGGL(pm_scatter_kernel<__half>, piece_blocks(a.s.i0), dim3(256), 0, st, a);
    else
      hipLaunchKernelGGL(pm_scatter_kernel<float>, piece_blocks(a.s.i0), dim3(256), 0, st, a);
    PFN_HIP(ctx, hipGetLastError());
  }
  PFN_HIP(ctx, hipStreamSynchronize(st));
  m.n = total;
  m.grid = G;
  m.n_bins = n_bins;
  for (int i = 0; i < 8; ++i) m.g_bins[i] = i < n_bins ? g_bins[i] : 0.0f;
  m.valid = true;
  return PFN_OK;
}

hipError_t pm_launch_estimate(pfn_context *ctx, const float *xyz, const float *dir,
                              const int32_t *bin, int64_t n, float radius, int k, float *out,
                              float *r_out, int32_t *n_out, hipStream_t st) {
  const PhotonMapState &m = ctx->pmap;
  PmEstArgs a{};
  a.ra = m.ra;
  a.rb = m.rb;
  a.rc = m.rc;
  a.start = m.start;
  a.G = m.grid;
  a.n_bins = m.n_bins;
  for (int i = 0; i < 8; ++i) a.g_bins[i] = m.g_bins[i];
  a.qx = xyz;
  a.qw = dir;
  a.qbin = bin;
  a.n = n;
  a.radius = radius;
  a.k = k;
  a.out = out;
  a.r_out = r_out;
  a.n_out = n_out;
  // 64 work-items per query: at most PFN_DISPATCH_ITEMS / 64 queries per launch
  const int64_t piece = PFN_DISPATCH_ITEMS / 64;
  for (a.q0 = 0; a.q0 < n; a.q0 += piece) {
    const dim3 gr((unsigned)std::min<int64_t>(n - a.q0, piece));
    if (k > 0)
      hipLaunchKernelGGL(pm_estimate_kernel<true>, gr, dim3(64), 0, st, a);
    else
      hipLaunchKernelGGL(pm_estimate_kernel<false>, gr, dim3(64), 0, st, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

__global__ void pm_unpack_kernel(const float4 *__restrict__ ra, const float4 *__restrict__ rb,
                                 const float *__restrict__ rc, uint64_t i0, uint64_t n, float *pos,
                                 float *dir, float *score) {
  const uint64_t i = i0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 a = ra[i], b = rb[i];
  if (pos) {
    pos[3 * i] = a.x;
    pos[3 * i + 1] = a.y;
    pos[3 * i + 2] = a.z;
  }
  if (dir) {
    dir[3 * i] = b.x;
    dir[3 * i + 1] = b.y;
    dir[3 * i + 2] = b.z;
  }
  if (score) {
    score[3 * i] = a.w;
    score[3 * i + 1] = b.w;
    score[3 * i + 2] = rc[i];
  }
}

hipError_t pm_launch_unpack(pfn_context *ctx, float *pos, float *dir, float *score, uint64_t n) {
  const PhotonMapState &m = ctx->pmap;
  const uint64_t piece = (uint64_t)PFN_DISPATCH_ITEMS;
  for (uint64_t i0 = 0; i0 < n; i0 += piece) {
    const uint64_t c = std::min(n - i0, piece);
    hipLaunchKernelGGL(pm_unpack_kernel, dim3((unsigned)((c + 255) / 256)), dim3(256), 0,
                       ctx->stream, m.ra, m.rb, m.rc, i0, n, pos, dir, score);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
