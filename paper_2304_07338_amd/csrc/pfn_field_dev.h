// Photon field on gfx950: multi-resolution grid encodings (position 3-D, direction 2-D, g raw)
// and the ReLU MLP on the matrix cores, as device functions shared by the query, render and
// training kernels.
//
// Matrix-core layout.  A 16-query tile is one wave: the MLP runs transposed, out^T = W * in^T,
// with v_mfma_f32_16x16x32_{f16,bf16} (or 16x16x4 f32).  The accumulator of one 16x16 tile
// holds, in lane l, rows 4*(l/16)+r (r = 0..3) of column l%16, which is exactly the shape of the
// B operand of the next layer (k rows 8*(l/16)+i, column l%16) once two accumulator tiles are
// concatenated.  The K order that this induces is a fixed permutation of the neurons, and the
// same permutation is applied to the weights when they are packed into LDS, so activations
// never leave registers between layers.  The input layer's B operand is produced directly by
// the encoder: lane group q = l/16 computes grid levels 4q..4q+3 of query l%16.
#pragma once
#include "pfn_device.h"

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

enum Prec : int { P_F32 = 0, P_F16 = 1, P_BF16 = 2 };

#define PFN_MAX_LEVELS 16
#define PFN_MAX_HIDDEN 7
#define PFN_WIDTH 64

// Per-level constants of one grid encoding.
struct GridLevels {
  int res[PFN_MAX_LEVELS];
  uint32_t off[PFN_MAX_LEVELS];  // entry offset of the level inside its table
  uint32_t dense_mask;           // bit l: level l is a dense (unhashed) grid
};

struct FieldDev {
  GridLevels pos, dir;
  // An entry holds 2 * fg features: f32 tables fg float2 per entry, f16/bf16 tables fg 32-bit
  // words (2 packed 16-bit features each) per entry.
  const void *pos_table;
  const void *dir_table;
  uint32_t hash_mask;     // 2^log2_table - 1
  uint32_t pair_ok;       // bit 0 / 1: the position / direction table starts on a pair of entries
  int levels;
  int hidden;             // hidden layers
  int fg;                 // feature groups: features per level / 2 (1 or 4)
  float psi, kappa;
};

// Sizes (in elements) of the packed MLP image in LDS order.  The input layer has, per 16-row
// tile, fg position chunks, fg direction chunks and one g chunk (16-bit: K = 32 per chunk; FP32:
// 8 K = 4 chunks per feature group and kind, and one for g).
__host__ __device__ constexpr int mlp_packed_elems(int prec, int hidden, int fg = 1) {
  return prec == P_F32 ? (4 * (16 * fg + 1) * 64 + (hidden - 1) * 4 * 16 * 64 + 16 * 64)
                       : (4 * (2 * fg + 1) * 64 * 8 + (hidden - 1) * 4 * 2 * 64 * 8 + 2 * 64 * 8);
}

// ------------------------------------------------------------------ encoding
// The spatial hash of Mueller et al. (2022), Section 3: XOR of coordinate * prime.
__device__ __forceinline__ uint32_t hash3(uint32_t x, uint32_t y, uint32_t z) {
  return x ^ (y * 2654435761u) ^ (z * 805459861u);
}
__device__ __forceinline__ uint32_t hash2(uint32_t x, uint32_t y) { return x ^ (y * 2654435761u); }

// Cell index and fraction of x in [0,1] on a level of resolution N: c = min(floor(xN), N-1),
// f = xN - c computed with one rounding (fma) so that fine levels keep full precision.
__device__ __forceinline__ void level_cell(float x, int N, int &c, float &f) {
  float y = x * (float)N;
  float fl = fminf(floorf(y), (float)(N - 1));
  c = (int)fl;
  f = fmaf(x, (float)N, -fl);
}

template <int P>
__device__ __forceinline__ float2 unpack_feat(uint32_t v) {
  if constexpr (P == P_F16) {
    __half2 h = *reinterpret_cast<__half2 *>(&v);
    return __half22float2(h);
  } else {
    return make_float2(__uint_as_float(v << 16), __uint_as_float(v & 0xFFFF0000u));
  }
}

template <int P>
__device__ __forceinline__ float2 load_feat(const void *table, uint32_t e) {
  if constexpr (P == P_F32) {
    return reinterpret_cast<const float2 *>(table)[e];
  } else {
    return unpack_feat<P>(reinterpret_cast<const uint32_t *>(table)[e]);
  }
}

// Features of the entries e0 and e1 of the two x-neighbours of a cell edge.  When they form one
// aligned pair of entries, one wide load fetches both: on a hashed level that is every even x
// (the first hash prime is 1, so the two indices differ in bit 0 only), on a dense level every
// even e0.  Halving the loads matters on the fine hashed levels, where every corner pair is a
// separate cache line.
template <int P>
__device__ __forceinline__ void load_feat_pair(const void *table, bool pair_ok, uint32_t e0,
                                               uint32_t e1, float2 &v0, float2 &v1) {
  if (pair_ok && (e0 ^ e1) == 1u) {
    const bool swap = (e0 & 1u) != 0u;
    if constexpr (P == P_F32) {
      const float4 pr = reinterpret_cast<const float4 *>(table)[e0 >> 1];
      const float2 lo = make_float2(pr.x, pr.y), hi = make_float2(pr.z, pr.w);
      v0 = swap ? hi : lo;
      v1 = swap ? lo : hi;
    } else {
      const uint2 pr = reinterpret_cast<const uint2 *>(table)[e0 >> 1];
      v0 = unpack_feat<P>(swap ? pr.y : pr.x);
      v1 = unpack_feat<P>(swap ? pr.x : pr.y);
    }
  } else {
    v0 = load_feat<P>(table, e0);
    v1 = load_feat<P>(table, e1);
  }
}

// Level `lv` of the position grid at x: 2 interpolated features.
template <int P>
__device__ __forceinline__ float2 encode_pos_level(const FieldDev &F, int lv, f3 x) {
  int N = F.pos.res[lv];
  uint32_t off = F.pos.off[lv];
  bool dense = (F.pos.dense_mask >> lv) & 1u;
  int cx, cy, cz;
  float fx, fy, fz;
  level_cell(x.x, N, cx, fx);
  level_cell(x.y, N, cy, fy);
  level_cell(x.z, N, cz, fz);
  float2 acc = make_float2(0.0f, 0.0f);
  uint32_t s1 = (uint32_t)(N + 1), s2 = s1 * s1;
  const bool pair_ok = (F.pair_ok & 1u) != 0u;
  const float gx = 1.0f - fx;
#pragma unroll
  for (int k = 0; k < 8; k += 2) {  // corners k (x0) and k+1 (x1) share y and z
    uint32_t vx = (uint32_t)cx, vy = (uint32_t)(cy + ((k >> 1) & 1)),
             vz = (uint32_t)(cz + ((k >> 2) & 1));
    uint32_t i0 = dense ? (vx + vy * s1 + vz * s2) : (hash3(vx, vy, vz) & F.hash_mask);
    uint32_t i1 = dense ? (i0 + 1u) : (hash3(vx + 1u, vy, vz) & F.hash_mask);
    float wy = ((k >> 1) & 1) ? fy : 1.0f - fy, wz = ((k >> 2) & 1) ? fz : 1.0f - fz;
    float2 v0, v1;
    load_feat_pair<P>(F.pos_table, pair_ok, off + i0, off + i1, v0, v1);
    float w0 = gx * wy * wz, w1 = fx * wy * wz;
    acc.x = fmaf(w0, v0.x, acc.x);
    acc.y = fmaf(w0, v0.y, acc.y);
    acc.x = fmaf(w1, v1.x, acc.x);
    acc.y = fmaf(w1, v1.y, acc.y);
  }
  return acc;
}

template <int P>
__device__ __forceinline__ float2 encode_dir_level(const FieldDev &F, int lv, float u0, float u1) {
  int N = F.dir.res[lv];
  uint32_t off = F.dir.off[lv];
  bool dense = (F.dir.dense_mask >> lv) & 1u;
  int cx, cy;
  float fx, fy;
  level_cell(u0, N, cx, fx);
  level_cell(u1, N, cy, fy);
  float2 acc = make_float2(0.0f, 0.0f);
  uint32_t s1 = (uint32_t)(N + 1);
  const bool pair_ok = (F.pair_ok & 2u) != 0u;
#pragma unroll
  for (int k = 0; k < 4; k += 2) {  // corners k (x0) and k+1 (x1) share y
    uint32_t vx = (uint32_t)cx, vy = (uint32_t)(cy + ((k >> 1) & 1));
    uint32_t i0 = dense ? (vx + vy * s1) : (hash2(vx, vy) & F.hash_mask);
    uint32_t i1 = dense ? (i0 + 1u) : (hash2(vx + 1u, vy) & F.hash_mask);
    float wy = ((k >> 1) & 1) ? fy : 1.0f - fy;
    float2 v0, v1;
    load_feat_pair<P>(F.dir_table, pair_ok, off + i0, off + i1, v0, v1);
    float w0 = (1.0f - fx) * wy, w1 = fx * wy;
    acc.x = fmaf(w0, v0.x, acc.x);
    acc.y = fmaf(w0, v0.y, acc.y);
    acc.x = fmaf(w1, v1.x, acc.x);
    acc.y = fmaf(w1, v1.y, acc.y);
  }
  return acc;
}

// ---------------- 8 features per level (4 feature groups): one entry is 16 bytes at 16 bits
// (one load per corner) or 32 bytes in FP32 (two loads).
template <int P>
__device__ __forceinline__ void load_feat8(const void *table, uint32_t e, float v[8]) {
  if constexpr (P == P_F32) {
    const float4 a = reinterpret_cast<const float4 *>(table)[2 * (size_t)e];
    const float4 b = reinterpret_cast<const float4 *>(table)[2 * (size_t)e + 1];
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else {
    const uint4 w = reinterpret_cast<const uint4 *>(table)[e];
    const float2 f0 = unpack_feat<P>(w.x), f1 = unpack_feat<P>(w.y), f2 = unpack_feat<P>(w.z),
                 f3v = unpack_feat<P>(w.w);
    v[0] = f0.x; v[1] = f0.y; v[2] = f1.x; v[3] = f1.y;
    v[4] = f2.x; v[5] = f2.y; v[6] = f3v.x; v[7] = f3v.y;
  }
}

// Level `lv` of the position grid at x, 8 features.
template <int P>
__device__ __forceinline__ void encode_pos_level8(const FieldDev &F, int lv, f3 x, float acc[8]) {
  const int N = F.pos.res[lv];
  const uint32_t off = F.pos.off[lv];
  const bool dense = (F.pos.dense_mask >> lv) & 1u;
  int cx, cy, cz;
  float fx, fy, fz;
  level_cell(x.x, N, cx, fx);
  level_cell(x.y, N, cy, fy);
  level_cell(x.z, N, cz, fz);
  const uint32_t s1 = (uint32_t)(N + 1), s2 = s1 * s1;
#pragma unroll
  for (int f = 0; f < 8; ++f) acc[f] = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const uint32_t vx = (uint32_t)(cx + (k & 1)), vy = (uint32_t)(cy + ((k >> 1) & 1)),
                   vz = (uint32_t)(cz + ((k >> 2) & 1));
    const uint32_t idx = dense ? (vx + vy * s1 + vz * s2) : (hash3(vx, vy, vz) & F.hash_mask);
    const float w = ((k & 1) ? fx : 1.0f - fx) * (((k >> 1) & 1) ? fy : 1.0f - fy) *
                    (((k >> 2) & 1) ? fz : 1.0f - fz);
    float v[8];
    load_feat8<P>(F.pos_table, off + idx, v);
#pragma unroll
    for (int f = 0; f < 8; ++f) acc[f] = fmaf(w, v[f], acc[f]);
  }
}

// Level `lv` of the direction grid at (u0, u1), 8 features.
template <int P>
__device__ __forceinline__ void encode_dir_level8(const FieldDev &F, int lv, float u0, float u1,
                                                  float acc[8]) {
  const int N = F.dir.res[lv];
  const uint32_t off = F.dir.off[lv];
  const bool dense = (F.dir.dense_mask >> lv) & 1u;
  int cx, cy;
  float fx, fy;
  level_cell(u0, N, cx, fx);
  level_cell(u1, N, cy, fy);
  const uint32_t s1 = (uint32_t)(N + 1);
#pragma unroll
  for (int f = 0; f < 8; ++f) acc[f] = 0.0f;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t vx = (uint32_t)(cx + (k & 1)), vy = (uint32_t)(cy + ((k >> 1) & 1));
    const uint32_t idx = dense ? (vx + vy * s1) : (hash2(vx, vy) & F.hash_mask);
    const float w = ((k & 1) ? fx : 1.0f - fx) * (((k >> 1) & 1) ? fy : 1.0f - fy);
    float v[8];
    load_feat8<P>(F.dir_table, off + idx, v);
#pragma unroll
    for (int f = 0; f < 8; ++f) acc[f] = fmaf(w, v[f], acc[f]);
  }
}

// Normalised spherical coordinates (theta/pi, (phi+pi)/(2pi)) of a unit direction, in FP32.
// The cell and fraction on a direction level then come from level_cell's single-rounding
// split.  An error of a few ulps in the coordinate (acosf, atan2f and the scaling each round
// once) moves the fraction of a level with N cells by N times that error, about 5e-4 on the
// finest level of the standard field (N = 7006): the encoding itself is that sensitive to the
// direction, whose FP32 components carry the same relative rounding.
__device__ __forceinline__ void dir_coords(f3 w, float &u0, float &u1) {
  float z = fminf(1.0f, fmaxf(-1.0f, w.z));
  u0 = fminf(1.0f, fmaxf(0.0f, acosf(z) * (1.0f / PFN_PI)));
  u1 = fminf(1.0f, fmaxf(0.0f, (atan2f(w.y, w.x) + PFN_PI) * (0.5f / PFN_PI)));
}

__device__ __forceinline__ f3 clamp01(f3 x) {
  return {fminf(1.0f, fmaxf(0.0f, x.x)), fminf(1.0f, fmaxf(0.0f, x.y)),
          fminf(1.0f, fmaxf(0.0f, x.z))};
}

// The 16 encoder outputs of this lane for one query: pos[0..7] = position levels 4q..4q+3
// (2 features each), dir[0..7] = direction levels 4q..4q+3.  Levels >= F.levels give 0.
// With 16-bit tables every lane reads its four levels without branching (a level past the
// last, or an invalid query, reads level 0 and is zeroed), so that the compiler can put all of
// a lane's corner loads in flight together: the callers clamp x and the coordinates to [0,1],
// so every index is in range.  (With a branch per level the fused march kernel's 64-job batch
// took 1866 against 1606 ms.)  FP32 tables keep the branch: their wider loads in flight would
// spill the fused march kernel's registers.
template <int P>
__device__ __forceinline__ void encode_lane(const FieldDev &F, int q, f3 x, float u0, float u1,
                                            bool valid, float pos[8], float dir[8]) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int lv = 4 * q + j;
    const bool ok = valid && lv < F.levels;
    float2 a = make_float2(0.0f, 0.0f), b = make_float2(0.0f, 0.0f);
    if constexpr (P == P_F32) {
      if (ok) {
        a = encode_pos_level<P>(F, lv, x);
        b = encode_dir_level<P>(F, lv, u0, u1);
      }
    } else {
      const int lc = ok ? lv : 0;
      const float2 a0 = encode_pos_level<P>(F, lc, x);
      const float2 b0 = encode_dir_level<P>(F, lc, u0, u1);
      if (ok) {
        a = a0;
        b = b0;
      }
    }
    pos[2 * j] = a.x;
    pos[2 * j + 1] = a.y;
    dir[2 * j] = b.x;
    dir[2 * j + 1] = b.y;
  }
}

// The same for FG feature groups: pos[g][2j + f] / dir[g][2j + f] = feature 2g + f of
// level 4q + j.  FG = 1 is encode_lane.
template <int P, int FG>
__device__ __forceinline__ void encode_lane_g(const FieldDev &F, int q, f3 x, float u0, float u1,
                                              bool valid, float (&pos)[FG][8],
                                              float (&dir)[FG][8]) {
  if constexpr (FG == 1) {
    encode_lane<P>(F, q, x, u0, u1, valid, pos[0], dir[0]);
  } else {
    static_assert(FG == 4, "feature groups: 1 or 4");
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int lv = 4 * q + j;
      float a[8], b[8];
#pragma unroll
      for (int f = 0; f < 8; ++f) a[f] = b[f] = 0.0f;
      if (valid && lv < F.levels) {
        encode_pos_level8<P>(F, lv, x, a);
        encode_dir_level8<P>(F, lv, u0, u1, b);
      }
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        pos[g][2 * j] = a[2 * g];
        pos[g][2 * j + 1] = a[2 * g + 1];
        dir[g][2 * j] = b[2 * g];
        dir[g][2 * j + 1] = b[2 * g + 1];
      }
    }
  }
}

// ------------------------------------------------------------------ matrix-core MLP
template <int P>
struct Mma;

template <>
struct Mma<P_F16> {
  typedef half8 vec;
  static __device__ __forceinline__ f32x4 mma(vec a, vec b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ vec pack(const float *v) {
    vec r;
#pragma unroll
    for (int i = 0; i < 8; ++i) r[i] = (_Float16)v[i];
    return r;
  }
};

template <>
struct Mma<P_BF16> {
  typedef bf16x8 vec;
  static __device__ __forceinline__ f32x4 mma(vec a, vec b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ vec pack(const float *v) {
    vec r;
#pragma unroll
    for (int i = 0; i < 8; ++i) r[i] = (__bf16)v[i];
    return r;
  }
};

__device__ __forceinline__ f32x4 relu4(f32x4 v) {
  return f32x4{fmaxf(v[0], 0.0f), fmaxf(v[1], 0.0f), fmaxf(v[2], 0.0f), fmaxf(v[3], 0.0f)};
}

// Forward pass of one 16-query tile at 16-bit precision, in two parts.  w: packed weights in
// LDS (vec units); b0 = position features, b1 = direction features, b2 = (g, 0, ...) for lane
// group 0.  The input layer adds the direction and g products first and the position product
// last, so that a caller whose tiles share b1 and b2 (one ray per column) computes the first
// part once and gets the same bits.
template <int P>
__device__ __forceinline__ void mlp_input16(const typename Mma<P>::vec *__restrict__ w,
                                            typename Mma<P>::vec b1, typename Mma<P>::vec b2,
                                            f32x4 pre[4]) {
  typedef Mma<P> M;
  const int l = lane_id();
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f32x4 a = {0.0f, 0.0f, 0.0f, 0.0f};
    a = M::mma(w[(mt * 3 + 1) * 64 + l], b1, a);
    pre[mt] = M::mma(w[(mt * 3 + 2) * 64 + l], b2, a);
  }
}

// Second part: the position product, the hidden layers and the output layer.  Returns the
// output tile: lanes 0..15 hold (L'_r, L'_g, L'_b, 0) of query l.
// Hidden layers 2..H and the output layer, from the first hidden layer's activations acc; wl
// points at the image of W_1.
template <int P>
__device__ __forceinline__ f32x4 mlp_tail16(const typename Mma<P>::vec *__restrict__ wl,
                                            int hidden, f32x4 acc[4]) {
  typedef Mma<P> M;
  typedef typename M::vec vec;
  const int l = lane_id();
  for (int h = 1; h < hidden; ++h) {
    float t0[8], t1[8];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      t0[r] = acc[0][r];
      t0[4 + r] = acc[1][r];
      t1[r] = acc[2][r];
      t1[4 + r] = acc[3][r];
    }
    vec h0 = M::pack(t0), h1 = M::pack(t1);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f32x4 a = {0.0f, 0.0f, 0.0f, 0.0f};
      a = M::mma(wl[(mt * 2 + 0) * 64 + l], h0, a);
      a = M::mma(wl[(mt * 2 + 1) * 64 + l], h1, a);
      acc[mt] = relu4(a);
    }
    wl += 8 * 64;
  }
  float t0[8], t1[8];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    t0[r] = acc[0][r];
    t0[4 + r] = acc[1][r];
    t1[r] = acc[2][r];
    t1[4 + r] = acc[3][r];
  }
  vec h0 = M::pack(t0), h1 = M::pack(t1);
  f32x4 out = {0.0f, 0.0f, 0.0f, 0.0f};
  out = M::mma(wl[0 * 64 + l], h0, out);
  out = M::mma(wl[1 * 64 + l], h1, out);
  return out;
}

template <int P>
__device__ __forceinline__ f32x4 mlp_rest16(const typename Mma<P>::vec *__restrict__ w, int hidden,
                                            typename Mma<P>::vec b0, const f32x4 pre[4]) {
  typedef Mma<P> M;
  const int l = lane_id();
  f32x4 acc[4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) acc[mt] = relu4(M::mma(w[(mt * 3 + 0) * 64 + l], b0, pre[mt]));
  return mlp_tail16<P>(w + 12 * 64, hidden, acc);
}

template <int P>
__device__ __forceinline__ f32x4 mlp_forward16(const typename Mma<P>::vec *__restrict__ w,
                                               int hidden, typename Mma<P>::vec b0,
                                               typename Mma<P>::vec b1, typename Mma<P>::vec b2) {
  f32x4 pre[4];
  mlp_input16<P>(w, b1, b2, pre);
  return mlp_rest16<P>(w, hidden, b0, pre);
}

// FP32 variant on v_mfma_f32_16x16x4f32: one K=4 chunk per instruction; chunk c of the input
// layer carries, in lane group q, position feature 8q+c (c < 8), direction feature 8q+c-8
// (c < 16) or g (c = 16, q = 0); hidden chunk (t, r) carries neuron 16t+4q+r.
__device__ __forceinline__ f32x4 mlp_tail16_f32(const float *__restrict__ wl, int hidden,
                                                f32x4 acc[4]) {
  const int l = lane_id();
  for (int h = 1; h < hidden; ++h) {
    f32x4 nxt[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f32x4 a = {0.0f, 0.0f, 0.0f, 0.0f};
      const float *wm = wl + mt * 16 * 64 + l;
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          a = __builtin_amdgcn_mfma_f32_16x16x4f32(wm[(t * 4 + r) * 64], acc[t][r], a, 0, 0, 0);
      nxt[mt] = relu4(a);
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) acc[mt] = nxt[mt];
    wl += 4 * 16 * 64;
  }
  f32x4 out = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      out = __builtin_amdgcn_mfma_f32_16x16x4f32(wl[(t * 4 + r) * 64 + l], acc[t][r], out, 0, 0, 0);
  return out;
}

__device__ __forceinline__ f32x4 mlp_forward16_f32(const float *__restrict__ w, int hidden,
                                                   const float pos[8], const float dir[8],
                                                   float gin) {
  const int l = lane_id();
  f32x4 acc[4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f32x4 a = {0.0f, 0.0f, 0.0f, 0.0f};
    const float *wm = w + mt * 17 * 64 + l;
#pragma unroll
    for (int c = 0; c < 8; ++c) a = __builtin_amdgcn_mfma_f32_16x16x4f32(wm[c * 64], pos[c], a, 0, 0, 0);
#pragma unroll
    for (int c = 0; c < 8; ++c)
      a = __builtin_amdgcn_mfma_f32_16x16x4f32(wm[(8 + c) * 64], dir[c], a, 0, 0, 0);
    a = __builtin_amdgcn_mfma_f32_16x16x4f32(wm[16 * 64], gin, a, 0, 0, 0);
    acc[mt] = relu4(a);
  }
  return mlp_tail16_f32(w + 4 * 17 * 64, hidden, acc);
}

// ---------------- FG feature groups (FG = 1: the functions above).  Per 16-row tile the input
// layer's 16-bit image holds C = 2 FG + 1 chunks (position groups, direction groups, g); the FP32
// image 16 FG + 1 chunks (8 per position group, 8 per direction group, g).
template <int P, int FG>
__device__ __forceinline__ void mlp_input16_g(const typename Mma<P>::vec *__restrict__ w,
                                              const typename Mma<P>::vec (&b1)[FG],
                                              typename Mma<P>::vec b2, f32x4 pre[4]) {
  if constexpr (FG == 1) {
    mlp_input16<P>(w, b1[0], b2, pre);
  } else {
    typedef Mma<P> M;
    constexpr int C = 2 * FG + 1;
    const int l = lane_id();
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f32x4 a = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int g = 0; g < FG; ++g) a = M::mma(w[(mt * C + FG + g) * 64 + l], b1[g], a);
      pre[mt] = M::mma(w[(mt * C + 2 * FG) * 64 + l], b2, a);
    }
  }
}

template <int P, int FG>
__device__ __forceinline__ f32x4 mlp_rest16_g(const typename Mma<P>::vec *__restrict__ w,
                                              int hidden, const typename Mma<P>::vec (&b0)[FG],
                                              const f32x4 pre[4]) {
  if constexpr (FG == 1) {
    return mlp_rest16<P>(w, hidden, b0[0], pre);
  } else {
    typedef Mma<P> M;
    constexpr int C = 2 * FG + 1;
    const int l = lane_id();
    f32x4 acc[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f32x4 a = pre[mt];
#pragma unroll
      for (int g = 0; g < FG; ++g) a = M::mma(w[(mt * C + g) * 64 + l], b0[g], a);
      acc[mt] = relu4(a);
    }
    return mlp_tail16<P>(w + 4 * C * 64, hidden, acc);
  }
}

template <int FG>
__device__ __forceinline__ f32x4 mlp_forward16_f32_g(const float *__restrict__ w, int hidden,
                                                     const float (&pos)[FG][8],
                                                     const float (&dir)[FG][8], float gin) {
  if constexpr (FG == 1) {
    return mlp_forward16_f32(w, hidden, pos[0], dir[0], gin);
  } else {
    constexpr int C = 16 * FG + 1;
    const int l = lane_id();
    f32x4 acc[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f32x4 a = {0.0f, 0.0f, 0.0f, 0.0f};
      const float *wm = w + mt * C * 64 + l;
#pragma unroll
      for (int g = 0; g < FG; ++g)
#pragma unroll
        for (int c = 0; c < 8; ++c)
          a = __builtin_amdgcn_mfma_f32_16x16x4f32(wm[(8 * g + c) * 64], pos[g][c], a, 0, 0, 0);
#pragma unroll
      for (int g = 0; g < FG; ++g)
#pragma unroll
        for (int c = 0; c < 8; ++c)
          a = __builtin_amdgcn_mfma_f32_16x16x4f32(wm[(8 * FG + 8 * g + c) * 64], dir[g][c], a, 0,
                                                   0, 0);
      a = __builtin_amdgcn_mfma_f32_16x16x4f32(wm[16 * FG * 64], gin, a, 0, 0, 0);
      acc[mt] = relu4(a);
    }
    return mlp_tail16_f32(w + 4 * C * 64, hidden, acc);
  }
}

// One 16-query tile: encode (lane group q computes levels 4q..4q+3 of query l%16) and run the
// MLP.  Returns the output tile (lanes 0..15: L' of query l).
template <int P>
__device__ __forceinline__ f32x4 field_tile16(const FieldDev &F, const void *__restrict__ lds_w,
                                              f3 x, float u0, float u1, float g, bool valid) {
  const int q = lane_id() >> 4;
  float pos[8], dir[8];
  encode_lane<P>(F, q, clamp01(x), u0, u1, valid, pos, dir);
  float gin = (q == 0) ? g : 0.0f;
  if constexpr (P == P_F32) {
    return mlp_forward16_f32(reinterpret_cast<const float *>(lds_w), F.hidden, pos, dir, gin);
  } else {
    typedef Mma<P> M;
    float gz[8] = {gin, 0, 0, 0, 0, 0, 0, 0};
    return mlp_forward16<P>(reinterpret_cast<const typename M::vec *>(lds_w), F.hidden,
                            M::pack(pos), M::pack(dir), M::pack(gz));
  }
}

template <int P, int FG>
__device__ __forceinline__ f32x4 field_tile16_g(const FieldDev &F, const void *__restrict__ lds_w,
                                                f3 x, float u0, float u1, float g, bool valid) {
  if constexpr (FG == 1) {
    return field_tile16<P>(F, lds_w, x, u0, u1, g, valid);
  } else {
    const int q = lane_id() >> 4;
    float pos[FG][8], dir[FG][8];
    encode_lane_g<P, FG>(F, q, clamp01(x), u0, u1, valid, pos, dir);
    const float gin = (q == 0) ? g : 0.0f;
    if constexpr (P == P_F32) {
      return mlp_forward16_f32_g<FG>(reinterpret_cast<const float *>(lds_w), F.hidden, pos, dir,
                                     gin);
    } else {
      typedef Mma<P> M;
      typedef typename M::vec vec;
      float gz[8] = {gin, 0, 0, 0, 0, 0, 0, 0};
      vec b0[FG], b1[FG];
#pragma unroll
      for (int gi = 0; gi < FG; ++gi) {
        b0[gi] = M::pack(pos[gi]);
        b1[gi] = M::pack(dir[gi]);
      }
      const vec *w = reinterpret_cast<const vec *>(lds_w);
      f32x4 pre[4];
      mlp_input16_g<P, FG>(w, b1, M::pack(gz), pre);
      return mlp_rest16_g<P, FG>(w, F.hidden, b0, pre);
    }
  }
}

// Copy the packed MLP image (global) into LDS with all threads of the block.
__device__ __forceinline__ void stage_weights(void *lds, const void *__restrict__ src, int bytes) {
  const int4 *s = reinterpret_cast<const int4 *>(src);
  int4 *d = reinterpret_cast<int4 *>(lds);
  for (int i = threadIdx.x; i < bytes / 16; i += blockDim.x) d[i] = s[i];
}

__device__ __forceinline__ float decode_lp(float lp, float psi, float kappa) {
  return kappa * exp10f(-psi * lp);
}
