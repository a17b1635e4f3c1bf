// Per-sample device helpers shared by the ray-march kernels (internal): light-volume fetch,
// shadow transmittance, direct light from the point lights and the photon-cache gather.
#pragma once
#include "march.h"

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ float4 tri_fetch4(const ushort4 *__restrict__ p, const Tri &t) {
  const int o[8] = {t.ox0 + t.oy0 + t.oz0, t.ox1 + t.oy0 + t.oz0, t.ox0 + t.oy1 + t.oz0,
                    t.ox1 + t.oy1 + t.oz0, t.ox0 + t.oy0 + t.oz1, t.ox1 + t.oy0 + t.oz1,
                    t.ox0 + t.oy1 + t.oz1, t.ox1 + t.oy1 + t.oz1};
  float gx = 1.0f - t.fx, gy = 1.0f - t.fy, gz = 1.0f - t.fz;
  const float w[8] = {gx * gy * gz,       t.fx * gy * gz,      gx * t.fy * gz,
                      t.fx * t.fy * gz,   gx * gy * t.fz,      t.fx * gy * t.fz,
                      gx * t.fy * t.fz,   t.fx * t.fy * t.fz};
  // one 8-byte load per texel (four binary16 channels)
  const uint2 *q = reinterpret_cast<const uint2 *>(p);
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const uint2 v = q[o[k]];
    acc.x = fmaf(w[k], __half2float(__ushort_as_half((unsigned short)(v.x & 0xFFFFu))), acc.x);
    acc.y = fmaf(w[k], __half2float(__ushort_as_half((unsigned short)(v.x >> 16))), acc.y);
    acc.z = fmaf(w[k], __half2float(__ushort_as_half((unsigned short)(v.y & 0xFFFFu))), acc.z);
    acc.w = fmaf(w[k], __half2float(__ushort_as_half((unsigned short)(v.y >> 16))), acc.w);
  }
  return acc;
}

// tri_fetch4 for up to 3 lights from the quad copy of the light volume (grid qg over the light
// grid g): per z plane one 24-byte entry holds channels 0-2 of the four (x, y) corner texels.
// Same corners, weights and sums as tri_fetch4; channel 3 is 0.
__device__ __forceinline__ float4 tri_fetch4_quad(const uint32_t *__restrict__ q,
                                                  const BrickGrid &qg, const BrickGrid &g, f3 x) {
  int i0, i1, j0, j1, k0, k1;
  float fx, fy, fz;
  tri_axis(x.x, g.nx, i0, i1, fx);
  tri_axis(x.y, g.ny, j0, j1, fy);
  tri_axis(x.z, g.nz, k0, k1, fz);
  const int64_t oxy = (int64_t)brick_ox(quad_axis(i0, i1, g.nx)) + brick_oy(qg, quad_axis(j0, j1, g.ny));
  const uint32_t *p0 = q + 6 * (oxy + brick_oz(qg, k0)), *p1 = q + 6 * (oxy + brick_oz(qg, k1));
  float gx = 1.0f - fx, gy = 1.0f - fy, gz = 1.0f - fz;
  const float w[8] = {gx * gy * gz,   fx * gy * gz,   gx * fy * gz,   fx * fy * gz,
                      gx * gy * fz,   fx * gy * fz,   gx * fy * fz,   fx * fy * fz};
  uint32_t d[12];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    d[i] = p0[i];
    d[6 + i] = p1[i];
  }
  auto h = [&](int e) {  // binary16 value e of the 24 (texel e / 3, channel e % 3)
    const uint32_t v = d[e >> 1];
    return __half2float(__ushort_as_half((unsigned short)((e & 1) ? (v >> 16) : (v & 0xFFFFu))));
  };
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    acc.x = fmaf(w[k], h(3 * k), acc.x);
    acc.y = fmaf(w[k], h(3 * k + 1), acc.y);
    acc.z = fmaf(w[k], h(3 * k + 2), acc.z);
  }
  return acc;
}

template <typename VT>
__device__ __forceinline__ float sigma_at(const MarchArgs &a, const float4 *tf, f3 x) {
  float rho = density_march(reinterpret_cast<const VT *>(a.vol), a.vg, a.qvol, a.qg, x);
  return tf_lookup(tf, rho).w * a.ext_scale;
}

// Exact shadow transmittance: midpoint march from x to the light, clipped to the cube.
template <typename VT>
__device__ float shadow_T(const MarchArgs &a, const float4 *tf, f3 x, f3 p, float step) {
  f3 v = p - x;
  float dist = sqrtf(dot(v, v));
  if (!(dist > 0.0f)) return 1.0f;
  f3 d = v * (1.0f / dist);
  float t0, t1;
  if (!clip_cube(x, d, t0, t1)) return 1.0f;
  float tend = fminf(t1, dist);
  if (!(tend > t0)) return 1.0f;
  float len = tend - t0, tau = 0.0f;
  for (int k = 0;; ++k) {
    float l = fminf(step, len - (float)k * step);
    if (!(l > 0.0f)) break;
    float t = t0 + (float)k * step + 0.5f * l;
    tau = fmaf(sigma_at<VT>(a, tf, x + d * t), l, tau);
  }
  return expf(-tau);
}

template <typename VT, int DIRECT>
__device__ __forceinline__ f3 direct_light(const MarchArgs &a, const MarchJob &job,
                                           const float4 *tf, f3 x, f3 wo) {
  f3 Ld = {0.0f, 0.0f, 0.0f};
  float4 tl = make_float4(1.f, 1.f, 1.f, 1.f);
  if constexpr (DIRECT == PFN_DIRECT_LIGHT_VOLUME)
    tl = a.lquad ? tri_fetch4_quad(a.lquad, a.lqg, a.lvg, x)
                 : tri_fetch4(a.lightvol, tri_setup(a.lvg, x));
  // HG phase (1 - g^2) / (4 pi) * d^(-3/2), d = 1 + g^2 - 2 g mu, and the inverse-square falloff,
  // all through reciprocal square roots (no divisions in the step loop)
  const float g = job.g;
  const float hg_c = (1.0f - g * g) * (0.25f / PFN_PI), hg_a = 1.0f + g * g, hg_b = 2.0f * g;
#pragma unroll
  for (int l = 0; l < PFN_MAX_LIGHTS; ++l) {
    if (l >= a.n_lights || !((job.light_mask >> l) & 1)) continue;
    f3 p = {a.light_pos[l][0], a.light_pos[l][1], a.light_pos[l][2]};
    f3 v = x - p;
    float ir = rsqrtf(dot(v, v));  // r > 0 unless a sample falls exactly on a light
    float mu = dot(v, wo) * ir;
    float rd = rsqrtf(fmaf(-hg_b, mu, hg_a));
    float T;
    if constexpr (DIRECT == PFN_DIRECT_LIGHT_VOLUME)
      T = l == 0 ? tl.x : l == 1 ? tl.y : l == 2 ? tl.z : tl.w;
    else
      T = shadow_T<VT>(a, tf, x, p, job.step);
    float k = hg_c * (rd * rd * rd) * T * (ir * ir);
    Ld = Ld + f3{a.light_int[l][0], a.light_int[l][1], a.light_int[l][2]} * k;
  }
  return Ld;
}

__device__ __forceinline__ f3 cache_gather(const MarchArgs &a, const MarchJob &job, f3 x) {
  BrickGrid g{a.cache_res, a.cache_res, a.cache_res, 0, 0};
  x = clamp01(x);
  int i0, i1, j0, j1, k0, k1;
  float fx, fy, fz;
  tri_axis(x.x, g.nx, i0, i1, fx);
  tri_axis(x.y, g.ny, j0, j1, fy);
  tri_axis(x.z, g.nz, k0, k1, fz);
  const int R = a.cache_res;
  const size_t cells = (size_t)R * R * R;
  f3 out = {0.f, 0.f, 0.f};
  for (int bi = 0; bi < 2; ++bi) {
    float wb = bi == 0 ? 1.0f - job.wbin : job.wbin;
    if (wb == 0.0f) continue;
    const float4 *c = a.cache + (size_t)(bi == 0 ? job.bin0 : job.bin1) * cells;
    f3 acc = {0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      int ix = (k & 1) ? i1 : i0, iy = (k & 2) ? j1 : j0, iz = (k & 4) ? k1 : k0;
      float w = ((k & 1) ? fx : 1.0f - fx) * ((k & 2) ? fy : 1.0f - fy) * ((k & 4) ? fz : 1.0f - fz);
      float4 v = c[((size_t)iz * R + iy) * R + ix];
      acc = acc + f3{v.x, v.y, v.z} * w;
    }
    out = out + acc * wb;
  }
  return out;
}
