// Photon field parameters and inference: initialisation, the 16-bit grid copies and packed MLP
// images used by the matrix-core kernels, and the batched query kernel (Eq. 2, decoded with
// Eq. 7).
#include "pfn_ctx.h"

#define QUERY_THREADS 256

// ------------------------------------------------------------------ initialisation
// Grid features U(-1e-4, 1e-4); weight matrix m ~ U(-a, a) with a = sqrt(6 / (fan_in + fan_out)).
struct InitArgs {
  float *p;
  size_t grid_floats;
  size_t w_off[PFN_MAX_HIDDEN + 2];  // float offsets; w_off[n_mats] = end
  int rows[PFN_MAX_HIDDEN + 1], cols[PFN_MAX_HIDDEN + 1];
  int n_mats;
  uint64_t seed;
};

__global__ void field_init_kernel(InitArgs a, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Philox r;
  r.init(a.seed, i, 10u);
  float u = r.next() * 2.0f - 1.0f;
  if (i < a.grid_floats) {
    a.p[i] = 1e-4f * u;
    return;
  }
  int m = 0;
  while (m + 1 < a.n_mats && i >= a.w_off[m + 1]) ++m;
  float lim = sqrtf(6.0f / (float)(a.rows[m] + a.cols[m]));
  a.p[i] = lim * u;
}

hipError_t launch_field_init(pfn_context *ctx, FieldSlot &f, uint64_t seed) {
  InitArgs a{};
  a.p = f.master;
  a.grid_floats = f.mlp_off;
  int nm = f.desc.hidden_layers + 1;
  for (int m = 0; m < nm; ++m) {
    a.w_off[m] = f.w_off[m];
    a.rows[m] = (m == nm - 1) ? 3 : f.desc.width;
    a.cols[m] = (m == 0) ? (2 * f.desc.feats_per_level * f.desc.levels + 1) : f.desc.width;
  }
  a.w_off[nm] = f.n_params;
  a.n_mats = nm;
  a.seed = seed;
  size_t n = f.n_params;
  hipLaunchKernelGGL(field_init_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     ctx->stream, a, n);
  return hipGetLastError();
}

// ------------------------------------------------------------------ low-precision copies
// One 32-bit word (two 16-bit features) per pair of consecutive FP32 features; an entry of 2 fg
// features is fg words.
template <int P>
__global__ void pack_grid_kernel(const float2 *__restrict__ master, uint32_t *__restrict__ lp,
                                 size_t entries) {
  size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= entries) return;
  float2 v = master[e];
  if constexpr (P == P_F16) {
    __half2 h = __floats2half2_rn(v.x, v.y);
    lp[e] = *reinterpret_cast<uint32_t *>(&h);
  } else {
    __bf16 a = (__bf16)v.x, b = (__bf16)v.y;
    uint16_t ua = __builtin_bit_cast(uint16_t, a), ub = __builtin_bit_cast(uint16_t, b);
    lp[e] = (uint32_t)ua | ((uint32_t)ub << 16);
  }
}

struct PackArgs {
  const float *w[PFN_MAX_HIDDEN + 1];  // weight matrices (row-major out x in)
  int hidden, levels, n_in;
  int fg;                              // feature groups (features per level / 2)
};

// Column of W_0 that feeds lane group q, slot i of the chunk of feature group grp of kind
// (0 position, 1 direction): feature 2 grp + (i & 1) of level 4q + i / 2 (-1: zero padding).
__device__ __forceinline__ int in_col_g(const PackArgs &a, int kind, int grp, int q, int i) {
  const int lv = 4 * q + (i >> 1), f = i & 1, F = 2 * a.fg;
  if (lv >= a.levels) return -1;
  return kind * F * a.levels + F * lv + 2 * grp + f;
}
// 16-bit input chunk c of a row tile: fg position groups, fg direction groups, then g.
__device__ __forceinline__ int in_col(const PackArgs &a, int c, int q, int i) {
  if (c < 2 * a.fg) return in_col_g(a, c / a.fg, c % a.fg, q, i);
  return (q == 0 && i == 0) ? a.n_in - 1 : -1;
}
// Neuron held by lane group q, slot i of hidden chunk c (two accumulator tiles per chunk).
__device__ __forceinline__ int hid_col(int c, int q, int i) {
  return i < 4 ? 32 * c + 4 * q + i : 32 * c + 16 + 4 * q + (i - 4);
}

template <int P>
__global__ void pack_mlp16_kernel(PackArgs a, void *out_v, int total) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  int i = idx & 7, l = (idx >> 3) & 63, blk = idx >> 9;  // blk: (matrix tile, chunk) pair
  int row = l & 15, q = l >> 4;
  float v = 0.0f;
  const int C = 2 * a.fg + 1;
  if (blk < 4 * C) {
    int mt = blk / C, c = blk % C;
    int col = in_col(a, c, q, i);
    if (col >= 0) v = a.w[0][(16 * mt + row) * a.n_in + col];
  } else {
    int rb = blk - 4 * C;
    int h = 1 + rb / 8;
    if (h < a.hidden) {
      int mt = (rb % 8) / 2, c = rb % 2;
      v = a.w[h][(16 * mt + row) * PFN_WIDTH + hid_col(c, q, i)];
    } else {
      int c = rb - (a.hidden - 1) * 8;
      if (row < 3) v = a.w[a.hidden][row * PFN_WIDTH + hid_col(c, q, i)];
    }
  }
  if constexpr (P == P_F16) {
    reinterpret_cast<_Float16 *>(out_v)[idx] = (_Float16)v;
  } else {
    reinterpret_cast<__bf16 *>(out_v)[idx] = (__bf16)v;
  }
}

__global__ void pack_mlp32_kernel(PackArgs a, float *out, int total) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  int l = idx & 63, blk = idx >> 6;
  int row = l & 15, q = l >> 4;
  float v = 0.0f;
  const int C = 16 * a.fg + 1;
  if (blk < 4 * C) {
    int mt = blk / C, c = blk % C;
    int col = -1;
    if (c < 16 * a.fg) {
      // 8 chunks per feature group and kind: chunk i carries slot i (feature 8q + i of the group)
      int kind = c / (8 * a.fg), grp = (c % (8 * a.fg)) >> 3, i = c & 7;
      col = in_col_g(a, kind, grp, q, i);
    } else if (q == 0) {
      col = a.n_in - 1;
    }
    if (col >= 0) v = a.w[0][(16 * mt + row) * a.n_in + col];
  } else {
    int rb = blk - 4 * C;
    int h = 1 + rb / 64;
    if (h < a.hidden) {
      int mt = (rb % 64) / 16, tr = rb % 16;
      int t = tr >> 2, r = tr & 3;
      v = a.w[h][(16 * mt + row) * PFN_WIDTH + 16 * t + 4 * q + r];
    } else {
      int tr = rb - (a.hidden - 1) * 64;
      int t = tr >> 2, r = tr & 3;
      if (row < 3) v = a.w[a.hidden][row * PFN_WIDTH + 16 * t + 4 * q + r];
    }
  }
  out[idx] = v;
}

// Only the MLP image (used when the 16-bit grid copy has been refreshed elsewhere).
hipError_t launch_field_pack_mlp(pfn_context *ctx, FieldSlot &f, int prec) {
  PackArgs a{};
  for (int m = 0; m <= f.desc.hidden_layers; ++m) a.w[m] = f.master + f.w_off[m];
  a.hidden = f.desc.hidden_layers;
  a.levels = f.desc.levels;
  a.fg = f.desc.feats_per_level / 2;
  a.n_in = 2 * f.desc.feats_per_level * f.desc.levels + 1;
  int total = mlp_packed_elems(prec, a.hidden, a.fg);
  unsigned blocks = (unsigned)((total + 255) / 256);
  if (prec == P_F32)
    hipLaunchKernelGGL(pack_mlp32_kernel, dim3(blocks), dim3(256), 0, ctx->stream, a,
                       (float *)f.mlp_packed[prec], total);
  else if (prec == P_BF16)
    hipLaunchKernelGGL(pack_mlp16_kernel<P_BF16>, dim3(blocks), dim3(256), 0, ctx->stream, a,
                       f.mlp_packed[prec], total);
  else
    hipLaunchKernelGGL(pack_mlp16_kernel<P_F16>, dim3(blocks), dim3(256), 0, ctx->stream, a,
                       f.mlp_packed[prec], total);
  return hipGetLastError();
}

hipError_t launch_field_pack(pfn_context *ctx, FieldSlot &f, int prec) {
  PackArgs a{};
  for (int m = 0; m <= f.desc.hidden_layers; ++m) a.w[m] = f.master + f.w_off[m];
  a.hidden = f.desc.hidden_layers;
  a.levels = f.desc.levels;
  a.fg = f.desc.feats_per_level / 2;
  a.n_in = 2 * f.desc.feats_per_level * f.desc.levels + 1;
  int total = mlp_packed_elems(prec, a.hidden, a.fg);
  if (prec == P_F32) {
    hipLaunchKernelGGL(pack_mlp32_kernel, dim3((total + 255) / 256), dim3(256), 0, ctx->stream, a,
                       (float *)f.mlp_packed[prec], total);
    return hipGetLastError();
  }
  // feature pairs of both grids (one 32-bit word each)
  size_t entries = (f.pos_entries + f.dir_entries) * (size_t)(f.desc.feats_per_level / 2);
  unsigned gb = (unsigned)((entries + 255) / 256);
  if (prec == P_F16) {
    hipLaunchKernelGGL(pack_grid_kernel<P_F16>, dim3(gb), dim3(256), 0, ctx->stream,
                       (const float2 *)f.master, f.lp_table[prec], entries);
    hipLaunchKernelGGL(pack_mlp16_kernel<P_F16>, dim3((total + 255) / 256), dim3(256), 0,
                       ctx->stream, a, f.mlp_packed[prec], total);
  } else {
    hipLaunchKernelGGL(pack_grid_kernel<P_BF16>, dim3(gb), dim3(256), 0, ctx->stream,
                       (const float2 *)f.master, f.lp_table[prec], entries);
    hipLaunchKernelGGL(pack_mlp16_kernel<P_BF16>, dim3((total + 255) / 256), dim3(256), 0,
                       ctx->stream, a, f.mlp_packed[prec], total);
  }
  return hipGetLastError();
}

FieldDev make_field_dev(const FieldSlot &f, int prec) {
  FieldDev F{};
  F.pos = f.pos;
  F.dir = f.dir;
  const int fg = f.desc.feats_per_level / 2;
  if (prec == P_F32) {
    F.pos_table = f.master;
    F.dir_table = f.master + 2 * fg * f.pos_entries;
  } else {
    F.pos_table = f.lp_table[prec];
    F.dir_table = f.lp_table[prec] + fg * f.pos_entries;
  }
  F.hash_mask = (uint32_t)((1ull << f.desc.log2_table) - 1);
  // wide loads of entry pairs need each table to start at a multiple of two entries (two
  // features per entry only; 8-feature entries are 16- or 32-byte loads of their own)
  const size_t pair_bytes = prec == P_F32 ? 16 : 8;
  F.pair_ok = fg != 1 ? 0u
                      : ((((uintptr_t)F.pos_table % pair_bytes) == 0 ? 1u : 0u) |
                         (((uintptr_t)F.dir_table % pair_bytes) == 0 ? 2u : 0u));
  F.levels = f.desc.levels;
  F.hidden = f.desc.hidden_layers;
  F.fg = fg;
  F.psi = f.desc.psi;
  F.kappa = (float)f.kappa;
  return F;
}

// ------------------------------------------------------------------ batched query
template <int P, int FG>
__global__ __launch_bounds__(QUERY_THREADS) void field_query_kernel(
    FieldDev F, const void *__restrict__ mlp, int mlp_bytes, const float *__restrict__ xyz,
    const float *__restrict__ dir, const float *__restrict__ g, int64_t n, float *__restrict__ lp,
    float *__restrict__ rgb) {
  extern __shared__ __align__(16) unsigned char lds_w[];
  stage_weights(lds_w, mlp, mlp_bytes);
  __syncthreads();
  const int lane = lane_id();
  const int64_t wave = (int64_t)blockIdx.x * (QUERY_THREADS / 64) + (threadIdx.x >> 6);
  const int64_t base = wave * 64;  // one group of 64 queries per wave
  if (base < n) {
#pragma unroll 1
    for (int j = 0; j < 4; ++j) {
      int64_t qi = base + 16 * j + (lane & 15);
      bool valid = qi < n;
      f3 x = {0.f, 0.f, 0.f}, w = {0.f, 0.f, 1.f};
      float gg = 0.f;
      if (valid) {
        x = {xyz[3 * qi], xyz[3 * qi + 1], xyz[3 * qi + 2]};
        w = {dir[3 * qi], dir[3 * qi + 1], dir[3 * qi + 2]};
        gg = g[qi];
      }
      float u0, u1;
      dir_coords(w, u0, u1);
      f32x4 out = field_tile16_g<P, FG>(F, lds_w, x, u0, u1, gg, valid);
      if (lane < 16 && valid) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          lp[3 * qi + c] = out[c];
          if (rgb) rgb[3 * qi + c] = decode_lp(out[c], F.psi, F.kappa);
        }
      }
    }
  }
}

hipError_t launch_field_query(pfn_context *ctx, const FieldSlot &f, int prec, const float *xyz,
                              const float *dir, const float *g, int64_t n, float *lp, float *rgb) {
  FieldDev F = make_field_dev(f, prec);
  const int fg = f.desc.feats_per_level / 2;
  int bytes = mlp_packed_elems(prec, f.desc.hidden_layers, fg) * (prec == P_F32 ? 4 : 2);
  auto kernel = [&]() {
    if (fg == 1)
      return prec == P_F32    ? field_query_kernel<P_F32, 1>
             : prec == P_BF16 ? field_query_kernel<P_BF16, 1>
                              : field_query_kernel<P_F16, 1>;
    return prec == P_F32    ? field_query_kernel<P_F32, 4>
           : prec == P_BF16 ? field_query_kernel<P_BF16, 4>
                            : field_query_kernel<P_F16, 4>;
  }();
  // one work-item per query; batches beyond one dispatch's reach go in pieces
  for (int64_t o = 0; o < n; o += PFN_DISPATCH_ITEMS) {
    const int64_t m = std::min<int64_t>(n - o, PFN_DISPATCH_ITEMS);
    const dim3 gr((unsigned)((m + QUERY_THREADS - 1) / QUERY_THREADS)), bl(QUERY_THREADS);
    hipLaunchKernelGGL(kernel, gr, bl, bytes, ctx->stream, F, f.mlp_packed[prec], bytes,
                       xyz + 3 * o, dir + 3 * o, g + o, m, lp + 3 * o, rgb ? rgb + 3 * o : nullptr);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
