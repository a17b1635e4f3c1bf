// Photon-field training (Section 3.5) on gfx950.
//
// One step = three kernels:
//  1. train_fb_kernel: per 16-sample tile (one wave), draw the batch (Section 3.3: uniform x,
//     uniform direction, g from the phase pool; target = Eq. (6) of the cache value / kappa),
//     encode, run the MLP forward on the matrix cores with activations kept in registers, take
//     the L2 residual, run the backward pass back to the encoder inputs with the transposed
//     weight images, and scatter the encoder gradients into the FP32 grid gradients with
//     atomics.  The per-sample layer inputs and output gradients are written out (16-bit,
//     neuron-major) for the weight gradients.
//  2. dw_kernel: the weight gradients dW = sum_n delta_n a_n^T as split-K matrix-core products
//     over the batch, added atomically into the FP32 gradient.
//  3. adam_kernel: bias-corrected Adam on the FP32 master parameters (every parameter, every
//     step), refreshing the 16-bit grid copy in the same pass and clearing the gradient.
// Gradients are formed from the unscaled residuals y - y* and scaled by 2 / (3 n) in Adam (the
// derivative of the mean over n samples and 3 channels), which keeps 16-bit deltas in range.
#include "pfn_ctx.h"

#define TRAIN_THREADS 256

// ------------------------------------------------------------------ batch generation
struct SampleSrc {
  uint64_t seed;
  int64_t step;
  const float4 *cache;
  int cache_res, n_bins;
  float g_bins[8];
  float inv_kappa, psi;
  int g_uniform;  // 1: g uniform over [g_0, g_last], targets interpolated in g between bins
  float g_span;   // g_last - g_0
};

__device__ __forceinline__ float log_target(float v, float psi) {
  // Eq. (6): -log10(v) / psi above the precision threshold 10^-psi, else 1
  return v > exp10f(-psi) ? -log10f(v) / psi : 1.0f;
}

__device__ __forceinline__ void gen_sample(const SampleSrc &s, int64_t i, f3 &x, f3 &w, float &g,
                                           int &bin, float tgt[3]) {
  Philox r;
  r.init(s.seed, ((uint64_t)s.step << 32) | (uint64_t)(uint32_t)i, STREAM_TRAIN);
  x.x = r.next();
  x.y = r.next();
  x.z = r.next();
  // u = (k + 1/2) 2^-23 (exact in FP32).  Pool batches: bin = floor(u * n_bins), in exact
  // integer arithmetic, and g its pool value.  Uniform-g batches: g = g_0 + u (g_last - g_0),
  // bin the lower of the two neighbouring bins and wb the weight of the upper one.
  uint32_t k = r.next_u32() >> 9;
  float wb = 0.0f;
  if (s.g_uniform) {
    const float u = (float)(2u * k + 1u) * 0x1p-24f;
    g = fmaf(u, s.g_span, s.g_bins[0]);
    bin = 0;
    while (bin + 2 < s.n_bins && g >= s.g_bins[bin + 1]) ++bin;
    wb = (g - s.g_bins[bin]) / (s.g_bins[bin + 1] - s.g_bins[bin]);
  } else {
    bin = (int)(((2ull * k + 1ull) * (uint64_t)s.n_bins) >> 24);
    g = s.g_bins[bin];
  }
  float u1 = r.next(), u2 = r.next();
  w = iso_dir(u1, u2);
  const int R = s.cache_res;
  int i0, i1, j0, j1, k0, k1;
  float fx, fy, fz;
  tri_axis(x.x, R, i0, i1, fx);
  tri_axis(x.y, R, j0, j1, fy);
  tri_axis(x.z, R, k0, k1, fz);
  float v0 = 0.f, v1 = 0.f, v2 = 0.f;
  for (int bi = 0; bi < (s.g_uniform ? 2 : 1); ++bi) {
    const float4 *c = s.cache + (size_t)(bin + bi) * R * R * R;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      int ix = (q & 1) ? i1 : i0, iy = (q & 2) ? j1 : j0, iz = (q & 4) ? k1 : k0;
      float wq = ((q & 1) ? fx : 1.0f - fx) * ((q & 2) ? fy : 1.0f - fy) * ((q & 4) ? fz : 1.0f - fz);
      float4 e = c[((size_t)iz * R + iy) * R + ix];
      a0 = fmaf(wq, e.x, a0);
      a1 = fmaf(wq, e.y, a1);
      a2 = fmaf(wq, e.z, a2);
    }
    const float wbin = s.g_uniform ? (bi ? wb : 1.0f - wb) : 1.0f;
    v0 = fmaf(wbin, a0, v0);
    v1 = fmaf(wbin, a1, v1);
    v2 = fmaf(wbin, a2, v2);
  }
  tgt[0] = log_target(v0 * s.inv_kappa, s.psi);
  tgt[1] = log_target(v1 * s.inv_kappa, s.psi);
  tgt[2] = log_target(v2 * s.inv_kappa, s.psi);
}

// Samples i0 .. n-1 (a piece of a batch that one dispatch cannot hold starts at i0 > 0).
__global__ void train_batch_kernel(SampleSrc s, int64_t i0, int64_t n, float *xyz, float *dir,
                                   float *g, int32_t *bin, float *tgt) {
  int64_t i = i0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  f3 x, w;
  float gg, t[3];
  int b;
  gen_sample(s, i, x, w, gg, b, t);
  if (xyz) {
    xyz[3 * i] = x.x;
    xyz[3 * i + 1] = x.y;
    xyz[3 * i + 2] = x.z;
  }
  if (dir) {
    dir[3 * i] = w.x;
    dir[3 * i + 1] = w.y;
    dir[3 * i + 2] = w.z;
  }
  if (g) g[i] = gg;
  if (bin) bin[i] = b;
  if (tgt) {
    tgt[3 * i] = t[0];
    tgt[3 * i + 1] = t[1];
    tgt[3 * i + 2] = t[2];
  }
}

// ------------------------------------------------------------------ backward weight images
// Transposed weights in matrix-core operand order:
//  lastT  : dh = W_H^T e      (4 row tiles x 1 K chunk; K = the 3 output channels)
//  hidT[k]: dh = W_k^T delta  (rows = inputs of W_k in natural order, K = outputs of W_k in the
//                              order the delta tiles are packed)
//  firstT : dz = W_0^T delta  (rows permuted so that lane group q receives the gradients of the
//                              encoder features it computed: tile 0/1 = position features
//                              8q..8q+7, tile 2/3 = direction features 8q..8q+7)
struct BwdPackArgs {
  const float *w[PFN_MAX_HIDDEN + 1];
  int hidden, levels, n_in;
  int fg;  // feature groups (features per level / 2)
};

// firstT has 4 row tiles per feature group: position slots 0-3 and 4-7, direction slots 0-3 and
// 4-7 of the group's lane-group layout.
__host__ __device__ constexpr int bwd_elems(int prec, int hidden, int fg = 1) {
  return prec == P_F32 ? (4 * 64 + (hidden - 1) * 4 * 16 * 64 + 4 * fg * 16 * 64)
                       : (4 * 64 * 8 + (hidden - 1) * 4 * 2 * 64 * 8 + 4 * fg * 2 * 64 * 8);
}

// Input column of W_0 whose gradient lands in row rho of row tile mt (-1: none).  Tile mt
// belongs to feature group mt / 4; within it, tiles 0/1 hold position slots 0-3 / 4-7 and tiles
// 2/3 direction slots 0-3 / 4-7, slot s of lane group qq being feature 2 grp + (s & 1) of level
// 4 qq + s / 2.
__device__ __forceinline__ int first_row_col(const BwdPackArgs &a, int mt, int rho) {
  const int grp = mt >> 2, sub = mt & 3;
  int qq = rho >> 2, r = rho & 3;
  int feat = 8 * qq + ((sub & 1) ? 4 : 0) + r;  // feature slot of lane group qq
  int lv = feat >> 1, f = feat & 1;
  if (lv >= a.levels) return -1;
  const int F = 2 * a.fg;
  return (sub < 2 ? 0 : F * a.levels) + F * lv + 2 * grp + f;
}
__device__ __forceinline__ int hid_col_b(int c, int q, int i) {
  return i < 4 ? 32 * c + 4 * q + i : 32 * c + 16 + 4 * q + (i - 4);
}

template <int P>
__global__ void pack_bwd16_kernel(BwdPackArgs a, void *out, int total) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  int i = idx & 7, l = (idx >> 3) & 63, blk = idx >> 9;
  int rho = l & 15, q = l >> 4;
  float v = 0.0f;
  const int H = a.hidden;
  if (blk < 4) {  // lastT
    int mt = blk;
    if (q == 0 && i < 3) v = a.w[H][i * PFN_WIDTH + 16 * mt + rho];
  } else if (blk < 4 + (H - 1) * 8) {  // hidT for layers 1..H-1
    int rb = blk - 4;
    int k = 1 + rb / 8, mt = (rb % 8) / 2, c = rb % 2;
    v = a.w[k][hid_col_b(c, q, i) * PFN_WIDTH + 16 * mt + rho];
  } else {  // firstT
    int rb = blk - 4 - (H - 1) * 8;
    int mt = rb / 2, c = rb % 2;
    int col = first_row_col(a, mt, rho);
    if (col >= 0) v = a.w[0][hid_col_b(c, q, i) * a.n_in + col];
  }
  if constexpr (P == P_F16) reinterpret_cast<_Float16 *>(out)[idx] = (_Float16)v;
  else reinterpret_cast<__bf16 *>(out)[idx] = (__bf16)v;
}

__global__ void pack_bwd32_kernel(BwdPackArgs a, float *out, int total) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  int l = idx & 63, blk = idx >> 6;
  int rho = l & 15, q = l >> 4;
  float v = 0.0f;
  const int H = a.hidden;
  if (blk < 4) {  // lastT: lane group q carries channel q
    int mt = blk;
    if (q < 3) v = a.w[H][q * PFN_WIDTH + 16 * mt + rho];
  } else if (blk < 4 + (H - 1) * 64) {
    int rb = blk - 4;
    int k = 1 + rb / 64, mt = (rb % 64) / 16, tr = rb % 16;
    int t = tr >> 2, r = tr & 3;
    v = a.w[k][(16 * t + 4 * q + r) * PFN_WIDTH + 16 * mt + rho];
  } else {
    int rb = blk - 4 - (H - 1) * 64;
    int mt = rb / 16, tr = rb % 16;
    int t = tr >> 2, r = tr & 3;
    int col = first_row_col(a, mt, rho);
    if (col >= 0) v = a.w[0][(16 * t + 4 * q + r) * a.n_in + col];
  }
  out[idx] = v;
}

hipError_t launch_field_pack_bwd(pfn_context *ctx, FieldSlot &f, int prec) {
  BwdPackArgs a{};
  for (int m = 0; m <= f.desc.hidden_layers; ++m) a.w[m] = f.master + f.w_off[m];
  a.hidden = f.desc.hidden_layers;
  a.levels = f.desc.levels;
  a.fg = f.desc.feats_per_level / 2;
  a.n_in = 2 * f.desc.feats_per_level * f.desc.levels + 1;
  int total = bwd_elems(prec, a.hidden, a.fg);
  unsigned blocks = (unsigned)((total + 255) / 256);
  if (prec == P_F32)
    hipLaunchKernelGGL(pack_bwd32_kernel, dim3(blocks), dim3(256), 0, ctx->stream, a,
                       (float *)f.mlp_bwd[prec], total);
  else if (prec == P_BF16)
    hipLaunchKernelGGL(pack_bwd16_kernel<P_BF16>, dim3(blocks), dim3(256), 0, ctx->stream, a,
                       f.mlp_bwd[prec], total);
  else
    hipLaunchKernelGGL(pack_bwd16_kernel<P_F16>, dim3(blocks), dim3(256), 0, ctx->stream, a,
                       f.mlp_bwd[prec], total);
  return hipGetLastError();
}

// ------------------------------------------------------------------ fused forward/backward
struct TrainArgs {
  FieldDev F;
  const void *fwd;  // packed forward weights (operand order)
  const void *bwd;  // packed transposed weights
  SampleSrc src;
  const float *in_xyz, *in_dir, *in_g, *in_tgt;  // used when samples are given
  int64_t n, ldn;   // samples, padded leading dimension (multiple of 32)
  float *grad_pos, *grad_dir;  // FP32 gradients of the grid tables (2 floats per entry)
  void *act;        // per-layer deltas and inputs, neuron-major [rows][ldn]
  int64_t delta_off[PFN_MAX_HIDDEN + 1], in_off[PFN_MAX_HIDDEN + 1];  // element offsets
  double *loss;     // accumulated sum of (weighted) squared residuals
  int rel_loss;     // 1: relative L2, residuals weighted by 1 / (y^2 + 0.01) (held constant)
};

template <typename T>
__device__ __forceinline__ T to_t(float v);
template <>
__device__ __forceinline__ _Float16 to_t<_Float16>(float v) {
  return (_Float16)v;
}
template <>
__device__ __forceinline__ __bf16 to_t<__bf16>(float v) {
  return (__bf16)v;
}
template <>
__device__ __forceinline__ float to_t<float>(float v) {
  return v;
}

template <int P>
struct ActT {
  typedef _Float16 type;
};
template <>
struct ActT<P_BF16> {
  typedef __bf16 type;
};
template <>
struct ActT<P_F32> {
  typedef float type;
};

// ------------------------------------------------------------------ encoder-gradient scatter
// The grid gradients take FP32 atomics, whose cost is set by the number of memory requests, not
// of lanes: lanes of one instruction that hit one 64-byte segment share a request.  A lane
// therefore does not scatter its own sample's corners (every lane a different segment); the wave
// stages its 16 samples' encoder gradients in LDS and scatters them with a lane mapping in which
// the floats of an x-neighbour corner pair (the features of corner x0, then of corner x1: one
// run on dense levels, and on hashed levels whenever x0 is even, since the hash's x prime is 1)
// come from consecutive lanes: 4 lanes per pair with 2 features per level, 16 with 8.
#define TRAIN_WAVES (TRAIN_THREADS / 64)

// Staged gradients of one wave: per sample, position features at F lv + c and direction
// features at 16 F + F lv + c (F = 2 FG features per level), padded against bank conflicts.
template <int FG>
struct StagedGrads {
  static constexpr int STRIDE = 64 * FG + 1;
  float dz[TRAIN_WAVES][16][STRIDE];
  float xu[TRAIN_WAVES][16][6];  // x, y, z, u0, u1, valid
};

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lane (q, nl) holds the gradients of sample nl for levels 4q..4q+3: position gp[g][2j + f] and
// direction gd[g][2j + f] of level 4q + j, feature 2g + f.
template <int FG>
__device__ __forceinline__ void stage_grid_grads(StagedGrads<FG> &S, int wv, int q, int nl,
                                                 bool valid, f3 x, float u0, float u1,
                                                 const float (&gp)[FG][8],
                                                 const float (&gd)[FG][8]) {
  constexpr int F = 2 * FG;
  float *d = S.dz[wv][nl];
#pragma unroll
  for (int g = 0; g < FG; ++g)
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int c = F * (4 * q + (s >> 1)) + 2 * g + (s & 1);
      d[c] = valid ? gp[g][s] : 0.0f;
      d[16 * F + c] = valid ? gd[g][s] : 0.0f;
    }
  if (q == 0) {
    float *c = S.xu[wv][nl];
    c[0] = x.x;
    c[1] = x.y;
    c[2] = x.z;
    c[3] = u0;
    c[4] = u1;
    c[5] = valid ? 1.0f : 0.0f;
  }
}

// One corner of level lv for a staged sample: entry index and trilinear (bilinear) weight.
__device__ __forceinline__ void pos_corner(const FieldDev &F, int lv, const float *xu, int xb,
                                           int cp, uint32_t &idx, float &w) {
  const int N = F.pos.res[lv];
  const bool dense = (F.pos.dense_mask >> lv) & 1u;
  int cx, cy, cz;
  float fx, fy, fz;
  level_cell(xu[0], N, cx, fx);
  level_cell(xu[1], N, cy, fy);
  level_cell(xu[2], N, cz, fz);
  const uint32_t vx = (uint32_t)(cx + xb), vy = (uint32_t)(cy + (cp & 1)),
                 vz = (uint32_t)(cz + (cp >> 1));
  const uint32_t s1 = (uint32_t)(N + 1), s2 = s1 * s1;
  idx = dense ? (vx + vy * s1 + vz * s2) : (hash3(vx, vy, vz) & F.hash_mask);
  w = (xb ? fx : 1.0f - fx) * ((cp & 1) ? fy : 1.0f - fy) * ((cp >> 1) ? fz : 1.0f - fz);
}
__device__ __forceinline__ void dir_corner(const FieldDev &F, int lv, const float *xu, int xb,
                                           int cp, uint32_t &idx, float &w) {
  const int N = F.dir.res[lv];
  const bool dense = (F.dir.dense_mask >> lv) & 1u;
  int cx, cy;
  float fx, fy;
  level_cell(xu[3], N, cx, fx);
  level_cell(xu[4], N, cy, fy);
  const uint32_t vx = (uint32_t)(cx + xb), vy = (uint32_t)(cy + cp);
  const uint32_t s1 = (uint32_t)(N + 1);
  idx = dense ? (vx + vy * s1) : (hash2(vx, vy) & F.hash_mask);
  w = (xb ? fx : 1.0f - fx) * (cp ? fy : 1.0f - fy);
}

template <int FG>
__device__ __forceinline__ void scatter_staged(const TrainArgs &a, const StagedGrads<FG> &S,
                                               int wv, int lane) {
  const FieldDev &F = a.F;
  constexpr int NF = 2 * FG;  // features per level
  // lanes per (level, sample): position 4 corner pairs x 2 corners x NF features, direction 2
  // pairs x 2 x NF; consecutive lanes run over the features, then the pair's two corners
  constexpr int PL = 8 * NF, DL = 4 * NF;
  {
    const int r = lane % PL, cp = r / (2 * NF), xb = (r / NF) & 1, feat = r % NF;
    const int sub = lane / PL;  // sample within the instruction
    constexpr int PER = 64 / PL;
#pragma unroll 1
    for (int it = 0; it < (16 / PER) * F.levels; ++it) {
      const int lv = it / (16 / PER), smp = PER * (it % (16 / PER)) + sub;
      const float *xu = S.xu[wv][smp];
      const float gv = S.dz[wv][smp][NF * lv + feat];
      if (xu[5] == 0.0f) continue;
      uint32_t idx;
      float w;
      pos_corner(F, lv, xu, xb, cp, idx, w);
      atomicAdd(a.grad_pos + (size_t)NF * (F.pos.off[lv] + idx) + feat, w * gv);
    }
  }
  {
    const int r = lane % DL, cp = r / (2 * NF), xb = (r / NF) & 1, feat = r % NF;
    const int sub = lane / DL;
    constexpr int PER = 64 / DL;
#pragma unroll 1
    for (int it = 0; it < (16 / PER) * F.levels; ++it) {
      const int lv = it / (16 / PER), smp = PER * (it % (16 / PER)) + sub;
      const float *xu = S.xu[wv][smp];
      const float gv = S.dz[wv][smp][16 * NF + NF * lv + feat];
      if (xu[5] == 0.0f) continue;
      uint32_t idx;
      float w;
      dir_corner(F, lv, xu, xb, cp, idx, w);
      atomicAdd(a.grad_dir + (size_t)NF * (F.dir.off[lv] + idx) + feat, w * gv);
    }
  }
}

// Row of the layer-0 input matrix (the network input index) of slot s of feature group g in lane
// group q: position features F lv + c, direction features F L + F lv + c, g at 2 F L.
template <int FG>
__device__ __forceinline__ int in_row(int L, int q, int g, int s, bool dir) {
  constexpr int F = 2 * FG;
  return (dir ? F * L : 0) + F * (4 * q + (s >> 1)) + 2 * g + (s & 1);
}

template <int P, int H, bool GEN, int FG>
__global__ __launch_bounds__(TRAIN_THREADS) void train_fb_kernel(TrainArgs a) {
  typedef typename ActT<P>::type T;
  // One 16-sample tile per wave and no loop over tiles: the weight operands are then not
  // loop-invariant, so the compiler streams them from cache instead of pinning them in registers.
  const int lane = lane_id(), q = lane >> 4, nl = lane & 15;
  const int wv = threadIdx.x >> 6;
  const int64_t tile = (int64_t)blockIdx.x * TRAIN_WAVES + wv;
  const int64_t ntiles = a.ldn / 16;
  const int L = a.F.levels;
  constexpr int NF = 2 * FG;
  T *act = reinterpret_cast<T *>(a.act);
  __shared__ StagedGrads<FG> S;
  double wave_loss = 0.0;
  if (tile < ntiles) {
    const int64_t i = tile * 16 + nl;
    const bool valid = i < a.n;
    f3 x = {0.f, 0.f, 0.f}, w = {0.f, 0.f, 1.f};
    float g = 0.f, tgt[3] = {0.f, 0.f, 0.f};
    if (valid) {
      if constexpr (GEN) {
        int b;
        gen_sample(a.src, i, x, w, g, b, tgt);
      } else {
        x = {a.in_xyz[3 * i], a.in_xyz[3 * i + 1], a.in_xyz[3 * i + 2]};
        w = {a.in_dir[3 * i], a.in_dir[3 * i + 1], a.in_dir[3 * i + 2]};
        g = a.in_g[i];
        tgt[0] = a.in_tgt[3 * i];
        tgt[1] = a.in_tgt[3 * i + 1];
        tgt[2] = a.in_tgt[3 * i + 2];
      }
    }
    x = clamp01(x);
    float u0, u1;
    dir_coords(w, u0, u1);
    float pos[FG][8], dir[FG][8];
    encode_lane_g<P, FG>(a.F, q, x, u0, u1, valid, pos, dir);
    const float gin = (q == 0) ? g : 0.0f;

    // layer-0 inputs (rows = network input index)
    {
      T *in0 = act + a.in_off[0];
#pragma unroll
      for (int gr = 0; gr < FG; ++gr)
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          int lv = 4 * q + (s >> 1);
          if (lv < L) {
            in0[(int64_t)in_row<FG>(L, q, gr, s, false) * a.ldn + i] =
                to_t<T>(valid ? pos[gr][s] : 0.f);
            in0[(int64_t)in_row<FG>(L, q, gr, s, true) * a.ldn + i] =
                to_t<T>(valid ? dir[gr][s] : 0.f);
          }
        }
      if (q == 0) in0[(int64_t)(2 * NF * L) * a.ldn + i] = to_t<T>(valid ? g : 0.f);
    }

    float e[3], lsum[3];
    f32x4 dz[4 * FG];  // gradients of the encoder outputs (firstT row tiles)
    if constexpr (P == P_F32) {
      const float *W = reinterpret_cast<const float *>(a.fwd);
      const float *B = reinterpret_cast<const float *>(a.bwd);
      constexpr int C = 16 * FG + 1;
      f32x4 hv[H][4];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        f32x4 c = {0.f, 0.f, 0.f, 0.f};
        const float *wm = W + mt * C * 64 + lane;
#pragma unroll
        for (int gr = 0; gr < FG; ++gr)
#pragma unroll
          for (int k = 0; k < 8; ++k)
            c = __builtin_amdgcn_mfma_f32_16x16x4f32(wm[(8 * gr + k) * 64], pos[gr][k], c, 0, 0, 0);
#pragma unroll
        for (int gr = 0; gr < FG; ++gr)
#pragma unroll
          for (int k = 0; k < 8; ++k)
            c = __builtin_amdgcn_mfma_f32_16x16x4f32(wm[(8 * FG + 8 * gr + k) * 64], dir[gr][k], c,
                                                     0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(wm[16 * FG * 64], gin, c, 0, 0, 0);
        hv[0][mt] = relu4(c);
      }
      const float *wl = W + 4 * C * 64;
#pragma unroll
      for (int k = 1; k < H; ++k) {
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
          f32x4 c = {0.f, 0.f, 0.f, 0.f};
          const float *wm = wl + mt * 16 * 64 + lane;
#pragma unroll
          for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              c = __builtin_amdgcn_mfma_f32_16x16x4f32(wm[(t * 4 + r) * 64], hv[k - 1][t][r], c, 0, 0, 0);
          hv[k][mt] = relu4(c);
        }
        wl += 4 * 16 * 64;
      }
      f32x4 out = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          out = __builtin_amdgcn_mfma_f32_16x16x4f32(wl[(t * 4 + r) * 64 + lane], hv[H - 1][t][r], out, 0, 0, 0);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float y = __shfl(out[c], nl);
        const float r = valid ? y - tgt[c] : 0.0f;
        const float wgt = a.rel_loss ? 1.0f / fmaf(y, y, 0.01f) : 1.0f;
        e[c] = r * wgt;
        lsum[c] = r * r * wgt;
      }
      // output layer: delta = e (rows = channels), input = h_{H-1}
      if (q == 0) {
        T *d = act + a.delta_off[H];
#pragma unroll
        for (int c = 0; c < 3; ++c) d[(int64_t)c * a.ldn + i] = to_t<T>(e[c]);
      }
      f32x4 acc[4];
      const float ec = q < 3 ? e[q] : 0.0f;
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        f32x4 c = {0.f, 0.f, 0.f, 0.f};
        acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(B[mt * 64 + lane], ec, c, 0, 0, 0);
      }
      const float *bh = B + 4 * 64;
#pragma unroll
      for (int k = H - 1; k >= 0; --k) {
        // inputs of layer k+1 (= h_k) and the output gradient of layer k
        T *ik = act + a.in_off[k + 1];
        T *dk = act + a.delta_off[k];
        T *ib = ik + (int64_t)(4 * q) * a.ldn + i;
        T *db = dk + (int64_t)(4 * q) * a.ldn + i;
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t ro = (int64_t)(16 * t + r) * a.ldn;  // row 16t + 4q + r
            float h = hv[k][t][r];
            acc[t][r] = h > 0.0f ? acc[t][r] : 0.0f;
            ib[ro] = to_t<T>(h);
            db[ro] = to_t<T>(acc[t][r]);
          }
        if (k >= 1) {
          const float *img = bh + (k - 1) * 4 * 16 * 64;
          f32x4 nxt[4];
#pragma unroll
          for (int mt = 0; mt < 4; ++mt) {
            f32x4 c = {0.f, 0.f, 0.f, 0.f};
            const float *wm = img + mt * 16 * 64 + lane;
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
              for (int r = 0; r < 4; ++r)
                c = __builtin_amdgcn_mfma_f32_16x16x4f32(wm[(t * 4 + r) * 64], acc[t][r], c, 0, 0, 0);
            nxt[mt] = c;
          }
#pragma unroll
          for (int mt = 0; mt < 4; ++mt) acc[mt] = nxt[mt];
        } else {
          const float *img = bh + (H - 1) * 4 * 16 * 64;  // firstT
#pragma unroll
          for (int mt = 0; mt < 4 * FG; ++mt) {
            f32x4 c = {0.f, 0.f, 0.f, 0.f};
            const float *wm = img + mt * 16 * 64 + lane;
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
              for (int r = 0; r < 4; ++r)
                c = __builtin_amdgcn_mfma_f32_16x16x4f32(wm[(t * 4 + r) * 64], acc[t][r], c, 0, 0, 0);
            dz[mt] = c;
          }
        }
      }
    } else {
      typedef Mma<P> M;
      typedef typename M::vec vec;
      constexpr int C = 2 * FG + 1;
      const vec *W = reinterpret_cast<const vec *>(a.fwd);
      const vec *B = reinterpret_cast<const vec *>(a.bwd);
      float gz[8] = {gin, 0, 0, 0, 0, 0, 0, 0};
      vec b0[FG], b1[FG];
#pragma unroll
      for (int gr = 0; gr < FG; ++gr) {
        b0[gr] = M::pack(pos[gr]);
        b1[gr] = M::pack(dir[gr]);
      }
      const vec b2 = M::pack(gz);
      vec hv[H][2];
      f32x4 acc[4];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int gr = 0; gr < FG; ++gr) c = M::mma(W[(mt * C + gr) * 64 + lane], b0[gr], c);
#pragma unroll
        for (int gr = 0; gr < FG; ++gr) c = M::mma(W[(mt * C + FG + gr) * 64 + lane], b1[gr], c);
        c = M::mma(W[(mt * C + 2 * FG) * 64 + lane], b2, c);
        acc[mt] = relu4(c);
      }
      const vec *wl = W + 4 * C * 64;
#pragma unroll
      for (int k = 0; k < H; ++k) {
        float t0[8], t1[8];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          t0[r] = acc[0][r];
          t0[4 + r] = acc[1][r];
          t1[r] = acc[2][r];
          t1[4 + r] = acc[3][r];
        }
        hv[k][0] = M::pack(t0);
        hv[k][1] = M::pack(t1);
        if (k + 1 < H) {
#pragma unroll
          for (int mt = 0; mt < 4; ++mt) {
            f32x4 c = {0.f, 0.f, 0.f, 0.f};
            c = M::mma(wl[(mt * 2 + 0) * 64 + lane], hv[k][0], c);
            c = M::mma(wl[(mt * 2 + 1) * 64 + lane], hv[k][1], c);
            acc[mt] = relu4(c);
          }
          wl += 8 * 64;
        }
      }
      f32x4 out = {0.f, 0.f, 0.f, 0.f};
      out = M::mma(wl[0 * 64 + lane], hv[H - 1][0], out);
      out = M::mma(wl[1 * 64 + lane], hv[H - 1][1], out);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float y = __shfl(out[c], nl);
        const float r = valid ? y - tgt[c] : 0.0f;
        const float wgt = a.rel_loss ? 1.0f / fmaf(y, y, 0.01f) : 1.0f;
        e[c] = r * wgt;
        lsum[c] = r * r * wgt;
      }
      if (q == 0) {
        T *d = act + a.delta_off[H];
#pragma unroll
        for (int c = 0; c < 3; ++c) d[(int64_t)c * a.ldn + i] = to_t<T>(e[c]);
      }
      float ev[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      if (q == 0) {
        ev[0] = e[0];
        ev[1] = e[1];
        ev[2] = e[2];
      }
      vec be = M::pack(ev);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        f32x4 c = {0.f, 0.f, 0.f, 0.f};
        acc[mt] = M::mma(B[mt * 64 + lane], be, c);
      }
      const vec *bh = B + 4 * 64;
#pragma unroll
      for (int k = H - 1; k >= 0; --k) {
        T *ik = act + a.in_off[k + 1];
        T *dk = act + a.delta_off[k];
        float dt[2][8];
        T *ib = ik + (int64_t)(4 * q) * a.ldn + i;
        T *db = dk + (int64_t)(4 * q) * a.ldn + i;
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int s = 0; s < 8; ++s) {
            int t = 2 * c + (s >> 2), r = s & 3;
            float h = (float)hv[k][c][s];
            float dv = h > 0.0f ? acc[t][r] : 0.0f;
            dt[c][s] = dv;
            const int64_t ro = (int64_t)(hid_col_b(c, 0, s)) * a.ldn;  // row hid_col(c, q, s)
            ib[ro] = hv[k][c][s];
            db[ro] = to_t<T>(dv);
          }
        vec bd0 = M::pack(dt[0]), bd1 = M::pack(dt[1]);
        if (k >= 1) {
          const vec *img = bh + (k - 1) * 8 * 64;
#pragma unroll
          for (int mt = 0; mt < 4; ++mt) {
            f32x4 c = {0.f, 0.f, 0.f, 0.f};
            c = M::mma(img[(mt * 2 + 0) * 64 + lane], bd0, c);
            c = M::mma(img[(mt * 2 + 1) * 64 + lane], bd1, c);
            acc[mt] = c;
          }
        } else {
          const vec *img = bh + (H - 1) * 8 * 64;  // firstT
#pragma unroll
          for (int mt = 0; mt < 4 * FG; ++mt) {
            f32x4 c = {0.f, 0.f, 0.f, 0.f};
            c = M::mma(img[(mt * 2 + 0) * 64 + lane], bd0, c);
            c = M::mma(img[(mt * 2 + 1) * 64 + lane], bd1, c);
            dz[mt] = c;
          }
        }
      }
    }
    {
      float gp[FG][8], gd[FG][8];
#pragma unroll
      for (int gr = 0; gr < FG; ++gr)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          gp[gr][r] = dz[4 * gr + 0][r];
          gp[gr][4 + r] = dz[4 * gr + 1][r];
          gd[gr][r] = dz[4 * gr + 2][r];
          gd[gr][4 + r] = dz[4 * gr + 3][r];
        }
      stage_grid_grads<FG>(S, wv, q, nl, valid, x, u0, u1, gp, gd);
    }
    wave_sync_lds();
    scatter_staged<FG>(a, S, wv, lane);
    if (q == 0) wave_loss += (double)lsum[0] + (double)lsum[1] + (double)lsum[2];
  }
  for (int off = 32; off > 0; off >>= 1) wave_loss += __shfl_down(wave_loss, off);
  if (lane == 0 && wave_loss != 0.0) atomicAdd(a.loss, wave_loss);
}

// ------------------------------------------------------------------ weight gradients
struct DwJob {
  int m, ot, it;
};
struct DwArgs {
  const void *act;
  int64_t ldn;
  int64_t delta_off, in_off;  // of this launch's layer
  int kchunk;                 // samples per wave
  int rows, cols;             // actual W_m size
  float *grad;                // W_m gradient (row-major rows x cols)
  int n_ot, n_it;
};

template <int P>
__global__ __launch_bounds__(64) void dw_kernel(DwArgs a) {
  typedef typename ActT<P>::type T;
  const int lane = lane_id(), q = lane >> 4, nl = lane & 15;
  const int tj = blockIdx.y;
  const int ot = tj / a.n_it, it = tj % a.n_it;
  const T *D = reinterpret_cast<const T *>(a.act) + a.delta_off + (int64_t)(16 * ot + nl) * a.ldn;
  const T *X = reinterpret_cast<const T *>(a.act) + a.in_off + (int64_t)(16 * it + nl) * a.ldn;
  const int64_t k0 = (int64_t)blockIdx.x * a.kchunk;
  int64_t k1 = k0 + a.kchunk;
  if (k1 > a.ldn) k1 = a.ldn;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  if constexpr (P == P_F32) {
    for (int64_t k = k0; k < k1; k += 4)
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(D[k + q], X[k + q], acc, 0, 0, 0);
  } else {
    typedef typename Mma<P>::vec vec;
    for (int64_t k = k0; k < k1; k += 32) {
      vec av = *reinterpret_cast<const vec *>(D + k + 8 * q);
      vec bv = *reinterpret_cast<const vec *>(X + k + 8 * q);
      acc = Mma<P>::mma(av, bv, acc);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    int o = 16 * ot + 4 * q + r, c = 16 * it + nl;
    if (o < a.rows && c < a.cols && acc[r] != 0.0f) atomicAdd(&a.grad[o * a.cols + c], acc[r]);
  }
}

// ------------------------------------------------------------------ Adam
struct AdamArgs {
  float *p, *m, *v, *g;
  size_t n, grid_floats;
  float lr, beta1, beta2, eps, bc1, bc2, gscale;
  uint32_t *lp16, *lpbf;  // optional 16-bit grid copies to refresh
};

__global__ void adam_kernel(AdamArgs a) {
  size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x;  // pair index
  size_t i0 = 2 * j;
  if (i0 >= a.n) return;
  float out[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    size_t i = i0 + s;
    if (i >= a.n) break;
    float g = a.g[i] * a.gscale;
    a.g[i] = 0.0f;
    float m = a.beta1 * a.m[i] + (1.0f - a.beta1) * g;
    float v = a.beta2 * a.v[i] + (1.0f - a.beta2) * g * g;
    a.m[i] = m;
    a.v[i] = v;
    float mh = m / a.bc1, vh = v / a.bc2;
    float p = a.p[i] - a.lr * mh / (sqrtf(vh) + a.eps);
    a.p[i] = p;
    out[s] = p;
  }
  if (i0 + 1 < a.grid_floats) {
    if (a.lp16) {
      __half2 h = __floats2half2_rn(out[0], out[1]);
      a.lp16[j] = *reinterpret_cast<uint32_t *>(&h);
    }
    if (a.lpbf) {
      __bf16 x = (__bf16)out[0], y = (__bf16)out[1];
      a.lpbf[j] = (uint32_t)__builtin_bit_cast(uint16_t, x) |
                  ((uint32_t)__builtin_bit_cast(uint16_t, y) << 16);
    }
  }
}

__global__ void scale_copy_kernel(const float *__restrict__ src, float *__restrict__ dst, size_t n,
                                  float s) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i] * s;
}

// ------------------------------------------------------------------ host side
struct TrainLayout {
  int64_t ldn;
  int64_t delta_off[PFN_MAX_HIDDEN + 1], in_off[PFN_MAX_HIDDEN + 1];
  int64_t elems;
};

// in0_rows: rows of the layer-0 input matrix (the network input padded to 16-row tiles)
static TrainLayout train_layout(int H, int64_t n, int in0_rows) {
  TrainLayout t{};
  t.ldn = (n + 31) / 32 * 32;
  int64_t off = 0;
  for (int m = 0; m <= H; ++m) {
    t.delta_off[m] = off;
    off += (int64_t)(m == H ? 16 : 64) * t.ldn;
  }
  for (int m = 0; m <= H; ++m) {
    t.in_off[m] = off;
    off += (int64_t)(m == 0 ? in0_rows : 64) * t.ldn;
  }
  t.elems = off;
  return t;
}

static int n_inputs(const FieldSlot &f) { return 2 * f.desc.feats_per_level * f.desc.levels + 1; }
static int in0_rows(const FieldSlot &f) { return std::max(80, (n_inputs(f) + 15) / 16 * 16); }

static pfn_status ensure_train_buffers(pfn_context *ctx, FieldSlot &f, int prec, int64_t n) {
  TrainLayout tl = train_layout(f.desc.hidden_layers, n, in0_rows(f));
  size_t bytes = (size_t)tl.elems * (prec == P_F32 ? 4 : 2);
  if (ctx->train_act_bytes < bytes) {
    if (ctx->train_act) (void)hipFree(ctx->train_act);
    ctx->train_act = nullptr;
    ctx->train_act_bytes = 0;
    PFN_HIP(ctx, hipMalloc(&ctx->train_act, bytes));
    ctx->train_act_bytes = bytes;
  }
  PFN_HIP(ctx, hipMemsetAsync(ctx->train_act, 0, bytes, ctx->stream));
  if (!f.mlp_bwd[prec]) {
    PFN_HIP(ctx, hipMalloc(&f.mlp_bwd[prec],
                           (size_t)bwd_elems(prec, f.desc.hidden_layers, f.desc.feats_per_level / 2) *
                               (prec == P_F32 ? 4 : 2)));
  }
  return PFN_OK;
}

static pfn_status refresh_train_images(pfn_context *ctx, FieldSlot &f, int prec) {
  pfn_status st = field_refresh(ctx, f, prec);
  if (st) return st;
  if (!f.bwd_valid[prec]) {
    PFN_HIP(ctx, launch_field_pack_bwd(ctx, f, prec));
    f.bwd_valid[prec] = true;
  }
  return PFN_OK;
}

template <int P, int H, bool GEN, int FG>
static hipError_t launch_fb_t(const TrainArgs &a, unsigned blocks, hipStream_t st) {
  hipLaunchKernelGGL((train_fb_kernel<P, H, GEN, FG>), dim3(blocks), dim3(TRAIN_THREADS), 0, st,
                     a);
  return hipGetLastError();
}
template <int P, bool GEN, int FG>
static hipError_t launch_fb_h(const TrainArgs &a, int H, unsigned blocks, hipStream_t st) {
  switch (H) {
    case 1: return launch_fb_t<P, 1, GEN, FG>(a, blocks, st);
    case 2: return launch_fb_t<P, 2, GEN, FG>(a, blocks, st);
    case 3: return launch_fb_t<P, 3, GEN, FG>(a, blocks, st);
    case 4: return launch_fb_t<P, 4, GEN, FG>(a, blocks, st);
    case 5: return launch_fb_t<P, 5, GEN, FG>(a, blocks, st);
    default: return hipErrorInvalidValue;
  }
}
template <bool GEN, int FG>
static hipError_t launch_fb_p(const TrainArgs &a, int prec, int H, unsigned blocks,
                              hipStream_t st) {
  if (prec == P_F32) return launch_fb_h<P_F32, GEN, FG>(a, H, blocks, st);
  if (prec == P_BF16) return launch_fb_h<P_BF16, GEN, FG>(a, H, blocks, st);
  return launch_fb_h<P_F16, GEN, FG>(a, H, blocks, st);
}
template <bool GEN>
static hipError_t launch_fb(const TrainArgs &a, int prec, int H, int fg, unsigned blocks,
                            hipStream_t st) {
  return fg == 1 ? launch_fb_p<GEN, 1>(a, prec, H, blocks, st)
                 : launch_fb_p<GEN, 4>(a, prec, H, blocks, st);
}

// Forward/backward over n samples into f.grad (unscaled), loss sum into *loss_dev.
static pfn_status run_fb(pfn_context *ctx, FieldSlot &f, int prec, int64_t n, bool gen,
                         const SampleSrc &src, const float *xyz, const float *dir, const float *g,
                         const float *tgt, double *loss_dev, int rel_loss) {
  const int H = f.desc.hidden_layers;
  const int fg = f.desc.feats_per_level / 2;
  TrainLayout tl = train_layout(H, n, in0_rows(f));
  TrainArgs a{};
  a.F = make_field_dev(f, prec);
  a.fwd = f.mlp_packed[prec];
  a.bwd = f.mlp_bwd[prec];
  a.src = src;
  a.in_xyz = xyz;
  a.in_dir = dir;
  a.in_g = g;
  a.in_tgt = tgt;
  a.n = n;
  a.ldn = tl.ldn;
  a.grad_pos = f.grad;
  a.grad_dir = f.grad + (size_t)f.desc.feats_per_level * f.pos_entries;
  a.act = ctx->train_act;
  for (int m = 0; m <= H; ++m) {
    a.delta_off[m] = tl.delta_off[m];
    a.in_off[m] = tl.in_off[m];
  }
  a.loss = loss_dev;
  a.rel_loss = rel_loss;
  int64_t ntiles = tl.ldn / 16;
  unsigned blocks = (unsigned)((ntiles + 3) / 4);
  const int tslot = timing_begin(ctx);
  PFN_HIP(ctx, gen ? launch_fb<true>(a, prec, H, fg, blocks, ctx->stream)
                   : launch_fb<false>(a, prec, H, fg, blocks, ctx->stream));
  timing_end(ctx, tslot, TK_TRAIN);
  // weight gradients, one launch per layer
  const int kchunk = 2048;
  for (int m = 0; m <= H; ++m) {
    DwArgs d{};
    d.act = ctx->train_act;
    d.ldn = tl.ldn;
    d.delta_off = tl.delta_off[m];
    d.in_off = tl.in_off[m];
    d.kchunk = kchunk;
    d.rows = m == H ? 3 : PFN_WIDTH;
    d.cols = m == 0 ? n_inputs(f) : PFN_WIDTH;
    d.grad = f.grad + f.w_off[m];
    d.n_ot = m == H ? 1 : 4;
    d.n_it = m == 0 ? in0_rows(f) / 16 : 4;
    dim3 grid((unsigned)((tl.ldn + kchunk - 1) / kchunk), (unsigned)(d.n_ot * d.n_it));
    if (prec == P_F32) hipLaunchKernelGGL(dw_kernel<P_F32>, grid, dim3(64), 0, ctx->stream, d);
    else if (prec == P_BF16) hipLaunchKernelGGL(dw_kernel<P_BF16>, grid, dim3(64), 0, ctx->stream, d);
    else hipLaunchKernelGGL(dw_kernel<P_F16>, grid, dim3(64), 0, ctx->stream, d);
    PFN_HIP(ctx, hipGetLastError());
  }
  return PFN_OK;
}

static pfn_status run_adam(pfn_context *ctx, FieldSlot &f, float *grad, int64_t t, float lr,
                           float b1, float b2, float eps, float gscale, int prec) {
  AdamArgs a{};
  a.p = f.master;
  a.m = f.adam_m;
  a.v = f.adam_v;
  a.g = grad;
  a.n = f.n_params;
  a.grid_floats = f.mlp_off;
  a.lr = lr;
  a.beta1 = b1;
  a.beta2 = b2;
  a.eps = eps;
  a.bc1 = (float)(1.0 - std::pow((double)b1, (double)t));
  a.bc2 = (float)(1.0 - std::pow((double)b2, (double)t));
  a.gscale = gscale;
  a.lp16 = prec == P_F16 ? f.lp_table[P_F16] : nullptr;
  a.lpbf = prec == P_BF16 ? f.lp_table[P_BF16] : nullptr;
  size_t pairs = (f.n_params + 1) / 2;
  const int tslot = timing_begin(ctx);
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, ctx->stream, a);
  PFN_HIP(ctx, hipGetLastError());
  timing_end(ctx, tslot, TK_ADAM);
  // The master changed: every derived copy is stale, except the 16-bit grid copy of the
  // training precision, which the Adam pass rewrote; its MLP image is repacked here.
  field_params_changed(f);
  if (prec != P_F32) {
    PFN_HIP(ctx, launch_field_pack_mlp(ctx, f, prec));
    f.lp_valid[prec] = true;
  }
  return PFN_OK;
}

static pfn_status check_training_field(pfn_context *ctx, FieldSlot &f) {
  if (!f.init) return pfn_fail(ctx, PFN_ERR_NOT_READY, "field not initialised");
  if (f.desc.hidden_layers > 5)
    return pfn_fail(ctx, PFN_ERR_UNSUPPORTED, "training supports 1 to 5 hidden layers");
  return PFN_OK;
}

static int prec_from(pfn_dtype d) { return d == PFN_F32 ? P_F32 : d == PFN_BF16 ? P_BF16 : P_F16; }

static SampleSrc make_src(pfn_context *ctx, uint64_t seed, int64_t step, float psi,
                          int g_sampling) {
  SampleSrc s{};
  s.seed = seed;
  s.step = step;
  s.cache = ctx->cache;
  s.cache_res = ctx->cache_res;
  s.n_bins = ctx->cache_bins;
  for (int b = 0; b < ctx->cache_bins; ++b) s.g_bins[b] = ctx->g_bins[b];
  s.inv_kappa = (float)(1.0 / ctx->kappa);
  s.psi = psi;
  s.g_uniform = (g_sampling == 1 && ctx->cache_bins > 1) ? 1 : 0;
  s.g_span = (float)((double)ctx->g_bins[ctx->cache_bins - 1] - (double)ctx->g_bins[0]);
  return s;
}

extern "C" pfn_status pfn_train_batch(pfn_context *ctx, uint64_t seed, int64_t step, int64_t n,
                                      int g_sampling, float *xyz, float *dir, float *g,
                                      int32_t *bin, float *tgt) {
  if (!ctx) return PFN_ERR_INVALID_ARG;
  if (g_sampling != 0 && g_sampling != 1)
    return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "g_sampling: 0 (pool) or 1 (uniform)");
  if (n < 0 || n > ((int64_t)1 << 32)) return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "n in [0, 2^32]");
  if (step < 0 || step >= ((int64_t)1 << 31))
    return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "step in [0, 2^31)");
  if (!ctx->cache_valid) return pfn_fail(ctx, PFN_ERR_NOT_READY, "no photon cache");
  if (n == 0) return PFN_OK;
  PFN_HIP(ctx, hipSetDevice(ctx->device));
  float psi = ctx->fields[ctx->cur_field].init ? ctx->fields[ctx->cur_field].desc.psi : 5.0f;
  SampleSrc s = make_src(ctx, seed, step, psi, g_sampling);
  for (int64_t o = 0; o < n; o += PFN_DISPATCH_ITEMS) {
    const int64_t m = std::min<int64_t>(n - o, PFN_DISPATCH_ITEMS);
    hipLaunchKernelGGL(train_batch_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0,
                       ctx->stream, s, o, o + m, xyz, dir, g, bin, tgt);
    PFN_HIP(ctx, hipGetLastError());
  }
  return PFN_OK;
}

extern "C" pfn_status pfn_field_forward_backward(pfn_context *ctx, pfn_dtype precision,
                                                 const float *xyz, const float *dir,
                                                 const float *g, const float *tgt, int64_t n,
                                                 int loss_mode, double *host_loss,
                                                 float *dev_grad) {
  if (!ctx) return PFN_ERR_INVALID_ARG;
  if (!(precision == PFN_F32 || precision == PFN_F16 || precision == PFN_BF16))
    return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "bad precision");
  if (n < 1 || n > ((int64_t)1 << 26)) return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "n in [1, 2^26]");
  if (!xyz || !dir || !g || !tgt) return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "NULL input");
  if (loss_mode != 0 && loss_mode != 1)
    return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "loss: 0 (L2) or 1 (relative L2)");
  FieldSlot &f = ctx->fields[ctx->cur_field];
  pfn_status st = check_training_field(ctx, f);
  if (st) return st;
  PFN_HIP(ctx, hipSetDevice(ctx->device));
  int prec = prec_from(precision);
  st = ensure_train_buffers(ctx, f, prec, n);
  if (st) return st;
  st = refresh_train_images(ctx, f, prec);
  if (st) return st;
  st = ensure_scratch(ctx, 64 * sizeof(double));
  if (st) return st;
  double *loss_dev = (double *)ctx->scratch;
  PFN_HIP(ctx, hipMemsetAsync(loss_dev, 0, sizeof(double), ctx->stream));
  PFN_HIP(ctx, hipMemsetAsync(f.grad, 0, f.n_params * 4, ctx->stream));
  SampleSrc src{};
  st = run_fb(ctx, f, prec, n, false, src, xyz, dir, g, tgt, loss_dev, loss_mode);
  if (st) return st;
  const float scale = (float)(2.0 / (3.0 * (double)n));
  if (dev_grad) {
    hipLaunchKernelGGL(scale_copy_kernel, dim3((unsigned)((f.n_params + 255) / 256)), dim3(256), 0,
                       ctx->stream, f.grad, dev_grad, f.n_params, scale);
    PFN_HIP(ctx, hipGetLastError());
  }
  double loss = 0.0;
  PFN_HIP(ctx, hipMemcpyAsync(&loss, loss_dev, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  PFN_HIP(ctx, hipMemsetAsync(f.grad, 0, f.n_params * 4, ctx->stream));
  PFN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (host_loss) *host_loss = loss / (3.0 * (double)n);
  if (!std::isfinite(loss)) return pfn_fail(ctx, PFN_ERR_NUMERIC, "loss is not finite");
  return PFN_OK;
}

extern "C" pfn_status pfn_field_adam_step(pfn_context *ctx, const float *dev_grad, int64_t t,
                                          float lr, float beta1, float beta2, float eps) {
  if (!ctx) return PFN_ERR_INVALID_ARG;
  if (!dev_grad) return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "gradient is NULL");
  if (t < 1) return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "t >= 1");
  if (!(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
      !(eps >= 0.0f))
    return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "bad Adam hyper-parameters");
  FieldSlot &f = ctx->fields[ctx->cur_field];
  if (!f.init) return pfn_fail(ctx, PFN_ERR_NOT_READY, "field not initialised");
  PFN_HIP(ctx, hipSetDevice(ctx->device));
  // the kernel clears the gradient it reads: work on a copy
  PFN_HIP(ctx, hipMemcpyAsync(f.grad, dev_grad, f.n_params * 4, hipMemcpyDeviceToDevice, ctx->stream));
  pfn_status st = run_adam(ctx, f, f.grad, t, lr, beta1, beta2, eps, 1.0f, P_F32);
  if (st) return st;
  f.adam_t = t;
  return PFN_OK;
}

__global__ void log_target_kernel(const float *__restrict__ v, float *__restrict__ tgt, int64_t n3,
                                  float inv_kappa, float psi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n3) tgt[i] = log_target(v[i] * inv_kappa, psi);
}

// Query radius of step s: the final radius, or the staggered schedule (fractions of Table 1).
static float step_radius(const pfn_train_params *p, int s) {
  if (!p->staggered) return p->radius;
  const double f = (double)s / (double)p->steps;
  const double r = f < 0.36 ? 0.125 : f < 0.63 ? 0.25 : f < 0.90 ? 0.5 : 1.0;
  return (float)(r * (double)p->radius);
}

extern "C" pfn_status pfn_train_step_radius(const pfn_train_params *p, int step, float *radius) {
  if (!p || !radius || p->steps < 1 || step < 0 || step >= p->steps) return PFN_ERR_INVALID_ARG;
  *radius = step_radius(p, step);
  return PFN_OK;
}

// Learning rate of step s (Section 3.5.1): constant, then decayed once at decay_start and once
// more every decay_interval steps.
static double step_lr(const pfn_train_params *p, int s) {
  double lr = p->lr;
  if (s >= p->decay_start)
    lr *= std::pow((double)p->decay, (double)(1 + (s - p->decay_start) / p->decay_interval));
  return lr;
}

extern "C" pfn_status pfn_train_lr_at(const pfn_train_params *p, int step, float *lr) {
  if (!p || !lr || p->steps < 1 || step < 0 || step >= p->steps || p->decay_interval < 1 ||
      p->decay_start < 0)
    return PFN_ERR_INVALID_ARG;
  *lr = (float)step_lr(p, step);
  return PFN_OK;
}

extern "C" pfn_status pfn_train_field(pfn_context *ctx, const pfn_train_params *p, float *hist) {
  if (!ctx) return PFN_ERR_INVALID_ARG;
  if (!p) return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "params are NULL");
  if (p->steps < 1 || p->steps > 1000000) return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "steps in [1, 1e6]");
  if (p->log2_batch < 4 || p->log2_batch > 22)
    return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "log2_batch in [4, 22]");
  if (!(p->lr > 0.0f) || !(p->beta1 >= 0.0f && p->beta1 < 1.0f) ||
      !(p->beta2 >= 0.0f && p->beta2 < 1.0f) || !(p->eps >= 0.0f) || !(p->decay > 0.0f) ||
      p->decay_interval < 1 || p->decay_start < 0)
    return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "bad optimiser hyper-parameters");
  if (!(p->precision == PFN_F32 || p->precision == PFN_F16 || p->precision == PFN_BF16))
    return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "bad precision");
  if (!ctx->cache_valid) return pfn_fail(ctx, PFN_ERR_NOT_READY, "no photon cache");
  if (p->target != 0 && p->target != 1)
    return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "target: 0 (cache) or 1 (photon map)");
  if (p->loss != 0 && p->loss != 1)
    return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "loss: 0 (L2) or 1 (relative L2)");
  if (p->g_sampling != 0 && p->g_sampling != 1)
    return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "g_sampling: 0 (pool) or 1 (uniform)");
  if (p->g_sampling == 1 && ctx->cache_bins < 2)
    return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "uniform g needs at least two cache bins");
  if (p->g_sampling == 1 && p->target != 0)
    return pfn_fail(ctx, PFN_ERR_UNSUPPORTED, "uniform g is supported for cache targets only");
  const bool map_targets = p->target == 1;
  if (map_targets) {
    if (!(std::isfinite(p->radius) && p->radius > 0.0f && p->radius <= 2.0f))
      return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "radius in (0, 2]");
    if (p->knn_k < 0 || p->knn_k > (1 << 20))
      return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "knn_k in [0, 2^20]");
    const PhotonMapState &m = ctx->pmap;
    if (!m.valid) return pfn_fail(ctx, PFN_ERR_NOT_READY, "no photon map");
    bool same = m.n_bins == ctx->cache_bins;
    for (int b = 0; same && b < m.n_bins; ++b) same = m.g_bins[b] == ctx->g_bins[b];
    if (!same) return pfn_fail(ctx, PFN_ERR_INVALID_ARG, "photon map and cache HG bins differ");
  }
  FieldSlot &f = ctx->fields[ctx->cur_field];
  pfn_status st = check_training_field(ctx, f);
  if (st) return st;
  PFN_HIP(ctx, hipSetDevice(ctx->device));
  const int prec = prec_from(p->precision);
  const int64_t n = (int64_t)1 << p->log2_batch;
  st = ensure_train_buffers(ctx, f, prec, n);
  if (st) return st;
  if (map_targets && ctx->pm_batch_cap < (size_t)n) {
    if (ctx->pm_batch) (void)hipFree(ctx->pm_batch);
    ctx->pm_batch = nullptr;
    ctx->pm_batch_cap = 0;
    // xyz, dir, value, target (3 floats each), g (1 float), bin (1 int)
    PFN_HIP(ctx, hipMalloc((void **)&ctx->pm_batch, sizeof(float) * 14 * (size_t)n));
    ctx->pm_batch_cap = (size_t)n;
  }
  float *b_xyz = ctx->pm_batch, *b_dir = b_xyz + 3 * n, *b_val = b_dir + 3 * n,
        *b_tgt = b_val + 3 * n, *b_g = b_tgt + 3 * n;
  int32_t *b_bin = reinterpret_cast<int32_t *>(b_g + n);
  st = ensure_scratch(ctx, sizeof(double) * (size_t)p->steps + 64);
  if (st) return st;
  double *loss_dev = (double *)ctx->scratch;
  PFN_HIP(ctx, hipMemsetAsync(loss_dev, 0, sizeof(double) * p->steps, ctx->stream));
  f.kappa = ctx->kappa;
  const float scale = (float)(2.0 / (3.0 * (double)n));
  for (int s = 0; s < p->steps; ++s) {
    st = refresh_train_images(ctx, f, prec);
    if (st) return st;
    SampleSrc src = make_src(ctx, p->seed, s, f.desc.psi, p->g_sampling);
    if (map_targets) {
      // the step's batch (the same samples as the cache targets would use), its Eq. (5)
      // estimates and their Eq. (6) encoding
      const unsigned nb = (unsigned)((n + 255) / 256);
      hipLaunchKernelGGL(train_batch_kernel, dim3(nb), dim3(256), 0, ctx->stream, src, 0, n, b_xyz,
                         b_dir, b_g, b_bin, nullptr);
      PFN_HIP(ctx, hipGetLastError());
      const int ts = timing_begin(ctx);
      PFN_HIP(ctx, pm_launch_estimate(ctx, b_xyz, b_dir, b_bin, n, step_radius(p, s), p->knn_k,
                                      b_val, nullptr, nullptr, ctx->stream));
      timing_end(ctx, ts, TK_PM_ESTIMATE);
      hipLaunchKernelGGL(log_target_kernel, dim3((unsigned)((3 * n + 255) / 256)), dim3(256), 0,
                         ctx->stream, b_val, b_tgt, 3 * n, src.inv_kappa, src.psi);
      PFN_HIP(ctx, hipGetLastError());
      st = run_fb(ctx, f, prec, n, false, src, b_xyz, b_dir, b_g, b_tgt, loss_dev + s, p->loss);
    } else {
      st = run_fb(ctx, f, prec, n, true, src, nullptr, nullptr, nullptr, nullptr, loss_dev + s,
                  p->loss);
    }
    if (st) return st;
    st = run_adam(ctx, f, f.grad, f.adam_t + 1, (float)step_lr(p, s), p->beta1, p->beta2, p->eps, scale, prec);
    if (st) return st;
    f.adam_t += 1;
  }
  std::vector<double> h(p->steps);
  PFN_HIP(ctx, hipMemcpyAsync(h.data(), loss_dev, sizeof(double) * p->steps,
                              hipMemcpyDeviceToHost, ctx->stream));
  PFN_HIP(ctx, hipStreamSynchronize(ctx->stream));
  bool finite = true;
  for (int s = 0; s < p->steps; ++s) {
    double l = h[s] / (3.0 * (double)n);
    if (hist) hist[s] = (float)l;
    finite &= std::isfinite(l);
  }
  if (!finite) return pfn_fail(ctx, PFN_ERR_NUMERIC, "training loss became NaN or Inf");
  return PFN_OK;
}
