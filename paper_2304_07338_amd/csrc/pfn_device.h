// Device-side building blocks shared by the gfx950 kernels: counter-based RNG, the
// Henyey-Greenstein phase function, unit-cube geometry, brick-ordered volume sampling and the
// transfer function.
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#define PFN_PI 3.14159265358979323846f

// ------------------------------------------------------------------ Philox4x32-10
// Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11).
struct Philox {
  uint32_t c0, c1, c2, c3;  // counter: item lo, item hi, stream id, block
  uint32_t k0, k1;          // key: seed lo, seed hi
  uint32_t b0, b1, b2, b3;  // current output block
  int pos;

  __device__ __forceinline__ void init(uint64_t seed, uint64_t item, uint32_t stream) {
    k0 = (uint32_t)seed;
    k1 = (uint32_t)(seed >> 32);
    c0 = (uint32_t)item;
    c1 = (uint32_t)(item >> 32);
    c2 = stream;
    c3 = 0;
    pos = 4;
  }
  __device__ __forceinline__ void block() {
    uint32_t x0 = c0, x1 = c1, x2 = c2, x3 = c3, y0 = k0, y1 = k1;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
      if (r) {
        y0 += 0x9E3779B9u;
        y1 += 0xBB67AE85u;
      }
      uint32_t hi0 = __umulhi(0xD2511F53u, x0), lo0 = 0xD2511F53u * x0;
      uint32_t hi1 = __umulhi(0xCD9E8D57u, x2), lo1 = 0xCD9E8D57u * x2;
      uint32_t n0 = hi1 ^ x1 ^ y0, n2 = hi0 ^ x3 ^ y1;
      x0 = n0;
      x1 = lo1;
      x2 = n2;
      x3 = lo0;
    }
    b0 = x0;
    b1 = x1;
    b2 = x2;
    b3 = x3;
    c3 += 1u;
    pos = 0;
  }
  __device__ __forceinline__ uint32_t next_u32() {
    if (pos == 4) block();
    uint32_t x = pos == 0 ? b0 : pos == 1 ? b1 : pos == 2 ? b2 : b3;
    ++pos;
    return x;
  }
  // Uniform in (0,1): ((x >> 9) + 1/2) * 2^-23, exact in binary32.
  __device__ __forceinline__ float next() {
    return ((float)(next_u32() >> 9) + 0.5f) * (1.0f / 8388608.0f);
  }
};

enum : uint32_t {
  STREAM_TRACE = 6,
  STREAM_TRAIN = 7,
  STREAM_RENDER = 8,
  STREAM_PT = 9,
  STREAM_FI_SAMPLE = 10,  // first-interaction renderer: free-flight walks along view rays
  STREAM_FI_NEE = 11      // first-interaction renderer: visibility walks toward the lights
};

// ------------------------------------------------------------------ small vector math
struct f3 {
  float x, y, z;
};
__device__ __forceinline__ f3 mk3(float x, float y, float z) { return f3{x, y, z}; }
__device__ __forceinline__ f3 operator+(f3 a, f3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ f3 operator-(f3 a, f3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ f3 operator*(f3 a, float s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ f3 mul(f3 a, f3 b) { return {a.x * b.x, a.y * b.y, a.z * b.z}; }
__device__ __forceinline__ float dot(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ f3 normalize3(f3 a) {
  float n = sqrtf(dot(a, a));
  return a * (1.0f / n);
}
__device__ __forceinline__ float maxc(f3 a) { return fmaxf(a.x, fmaxf(a.y, a.z)); }

// ------------------------------------------------------------------ Henyey-Greenstein
__device__ __forceinline__ float hg_eval(float g, float mu) {
  float d = 1.0f + g * g - 2.0f * g * mu;
  return (1.0f - g * g) / (4.0f * PFN_PI * d * sqrtf(d));
}

__device__ __forceinline__ float hg_sample_mu(float g, float u) {
  if (fabsf(g) < 1e-3f) return 1.0f - 2.0f * u;
  float sq = (1.0f - g * g) / (1.0f - g + 2.0f * g * u);
  float mu = (1.0f + g * g - sq * sq) / (2.0f * g);
  return fminf(1.0f, fmaxf(-1.0f, mu));
}

// New direction at cosine mu from w, azimuth 2 pi u2, in the orthonormal basis of Duff et al.,
// "Building an Orthonormal Basis, Revisited" (JCGT 2017).
__device__ __forceinline__ f3 hg_sample_dir(float g, f3 w, float u1, float u2) {
  float mu = hg_sample_mu(g, u1);
  float s = sqrtf(fmaxf(0.0f, 1.0f - mu * mu));
  float phi = 2.0f * PFN_PI * u2;
  float sign = w.z >= 0.0f ? 1.0f : -1.0f;
  float a = -1.0f / (sign + w.z);
  float b = w.x * w.y * a;
  f3 t1 = {1.0f + sign * w.x * w.x * a, sign * b, -sign * w.x};
  f3 t2 = {b, sign + w.y * w.y * a, -w.y};
  float sp, cp;
  sincosf(phi, &sp, &cp);
  f3 d = w * mu + (t1 * cp + t2 * sp) * s;
  return normalize3(d);
}

// Orthonormal basis around a unit vector (Duff et al., JCGT 2017).
__device__ __forceinline__ void onb(f3 w, f3 &t1, f3 &t2) {
  float sign = w.z >= 0.0f ? 1.0f : -1.0f;
  float a = -1.0f / (sign + w.z);
  float b = w.x * w.y * a;
  t1 = {1.0f + sign * w.x * w.x * a, sign * b, -sign * w.x};
  t2 = {b, sign + w.y * w.y * a, -w.y};
}

__device__ __forceinline__ f3 iso_dir(float u1, float u2);

// Photon emission from a point light p: uniform over the cone around the direction to the cube
// centre that contains the cube's bounding sphere (whole sphere if p is inside it).  Returns the
// cone's share of the full sphere, which scales the photon power (directions outside the cone
// cannot reach the cube).
__device__ __forceinline__ float emit_dir(f3 p, float u1, float u2, f3 &out) {
  f3 c = {0.5f - p.x, 0.5f - p.y, 0.5f - p.z};
  float d = sqrtf(dot(c, c));
  const float R = 0.86602540378443865f;
  if (!(d > R)) {
    out = iso_dir(u1, u2);
    return 1.0f;
  }
  f3 axis = c * (1.0f / d);
  float q = R / d;
  float cos_a = sqrtf(1.0f - q * q);
  float ct = 1.0f - u1 * (1.0f - cos_a);
  float st = sqrtf(fmaxf(0.0f, 1.0f - ct * ct));
  float sp, cp;
  sincosf(2.0f * PFN_PI * u2, &sp, &cp);
  f3 t1, t2;
  onb(axis, t1, t2);
  out = normalize3(axis * ct + (t1 * cp + t2 * sp) * st);
  return 0.5f * (1.0f - cos_a);
}

__device__ __forceinline__ f3 iso_dir(float u1, float u2) {
  float z = 1.0f - 2.0f * u1;
  float r = sqrtf(fmaxf(0.0f, 1.0f - z * z));
  float sp, cp;
  sincosf(2.0f * PFN_PI * u2, &sp, &cp);
  return {r * cp, r * sp, z};
}

// ------------------------------------------------------------------ unit cube geometry
__device__ __forceinline__ bool clip_cube(f3 o, f3 d, float &t0, float &t1) {
  float tn = -3.0e38f, tf = 3.0e38f;
  const float oo[3] = {o.x, o.y, o.z}, dd[3] = {d.x, d.y, d.z};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (dd[a] == 0.0f) {
      if (oo[a] < 0.0f || oo[a] > 1.0f) return false;
      continue;
    }
    float inv = 1.0f / dd[a];
    float ta = (0.0f - oo[a]) * inv, tb = (1.0f - oo[a]) * inv;
    tn = fmaxf(tn, fminf(ta, tb));
    tf = fminf(tf, fmaxf(ta, tb));
  }
  tn = fmaxf(tn, 0.0f);
  if (!(tn < tf)) return false;
  t0 = tn;
  t1 = tf;
  return true;
}

__device__ __forceinline__ float exit_distance(f3 x, f3 d) {
  float t = 3.0e38f;
  if (d.x > 0.0f) t = fminf(t, (1.0f - x.x) / d.x);
  else if (d.x < 0.0f) t = fminf(t, -x.x / d.x);
  if (d.y > 0.0f) t = fminf(t, (1.0f - x.y) / d.y);
  else if (d.y < 0.0f) t = fminf(t, -x.y / d.y);
  if (d.z > 0.0f) t = fminf(t, (1.0f - x.z) / d.z);
  else if (d.z < 0.0f) t = fminf(t, -x.z / d.z);
  return fmaxf(t, 0.0f);
}

// ------------------------------------------------------------------ brick-ordered grids
// Grids are stored in 8x8x8 bricks (512 elements), bricks in x-fastest order, elements inside a
// brick x-fastest.  A trilinear fetch splits its index into per-axis partial offsets, so the 8
// corner addresses cost 6 small products and 8 adds, and rays that march together touch the
// same 8^3 neighbourhoods.
struct BrickGrid {
  int nx, ny, nz;   // logical size
  int sy, sz;       // brick strides in elements for one brick step along y and z
};

__host__ __device__ __forceinline__ int brick_ox(int i) { return ((i >> 3) << 9) + (i & 7); }
__host__ __device__ __forceinline__ int brick_oy(const BrickGrid &g, int j) {
  return (j >> 3) * g.sy + ((j & 7) << 3);
}
__host__ __device__ __forceinline__ int brick_oz(const BrickGrid &g, int k) {
  return (k >> 3) * g.sz + ((k & 7) << 6);
}

// Trilinear interpolation over cell centres with clamp-to-edge: corner offsets and weights.
struct Tri {
  int ox0, ox1, oy0, oy1, oz0, oz1;
  float fx, fy, fz;
};
__device__ __forceinline__ void tri_axis(float x, int n, int &i0, int &i1, float &f) {
  const float u = fmaf(x, (float)n, -0.5f);  // one rounding, whatever the calling kernel
  float fl = floorf(u);
  f = u - fl;
  int lo = (int)fl;
  i0 = min(max(lo, 0), n - 1);
  i1 = min(max(lo + 1, 0), n - 1);
}
__device__ __forceinline__ Tri tri_setup(const BrickGrid &g, f3 x) {
  Tri t;
  int i0, i1, j0, j1, k0, k1;
  tri_axis(x.x, g.nx, i0, i1, t.fx);
  tri_axis(x.y, g.ny, j0, j1, t.fy);
  tri_axis(x.z, g.nz, k0, k1, t.fz);
  t.ox0 = brick_ox(i0);
  t.ox1 = brick_ox(i1);
  t.oy0 = brick_oy(g, j0);
  t.oy1 = brick_oy(g, j1);
  t.oz0 = brick_oz(g, k0);
  t.oz1 = brick_oz(g, k1);
  return t;
}

template <typename T>
__device__ __forceinline__ float to_f(T v);
template <>
__device__ __forceinline__ float to_f<float>(float v) {
  return v;
}
template <>
__device__ __forceinline__ float to_f<__half>(__half v) {
  return __half2float(v);
}

// Trilinear blend of the 8 corner values (x fastest), with the roundings spelled out so that
// every lookup form gives the same bits.
__device__ __forceinline__ float trilerp8(float c000, float c100, float c010, float c110,
                                          float c001, float c101, float c011, float c111,
                                          float fx, float fy, float fz) {
  const float gx = 1.0f - fx, gy = 1.0f - fy, gz = 1.0f - fz;
  const float c00 = fmaf(fx, c100, gx * c000), c10 = fmaf(fx, c110, gx * c010);
  const float c01 = fmaf(fx, c101, gx * c001), c11 = fmaf(fx, c111, gx * c011);
  const float c0 = fmaf(fy, c10, gy * c00), c1 = fmaf(fy, c11, gy * c01);
  return fmaf(fz, c1, gz * c0);
}

template <typename T>
__device__ __forceinline__ float tri_fetch(const T *__restrict__ p, const Tri &t) {
  return trilerp8(to_f(p[t.ox0 + t.oy0 + t.oz0]), to_f(p[t.ox1 + t.oy0 + t.oz0]),
                  to_f(p[t.ox0 + t.oy1 + t.oz0]), to_f(p[t.ox1 + t.oy1 + t.oz0]),
                  to_f(p[t.ox0 + t.oy0 + t.oz1]), to_f(p[t.ox1 + t.oy0 + t.oz1]),
                  to_f(p[t.ox0 + t.oy1 + t.oz1]), to_f(p[t.ox1 + t.oy1 + t.oz1]), t.fx, t.fy,
                  t.fz);
}

__device__ __forceinline__ bool inside_cube(f3 x) {
  return x.x >= 0.0f && x.x <= 1.0f && x.y >= 0.0f && x.y <= 1.0f && x.z >= 0.0f && x.z <= 1.0f;
}

template <typename T>
__device__ __forceinline__ float density_at(const T *__restrict__ vol, const BrickGrid &g, f3 x) {
  if (!inside_cube(x)) return 0.0f;
  return tri_fetch(vol, tri_setup(g, x));
}

// Index of the quad copy of a binary16 volume along x or y: the cell's lower corner plus one
// (0 .. n), recovered from the clamped corners of tri_axis (lower corner -1 gives 0 0, n-1
// gives n-1 n-1).
__device__ __forceinline__ int quad_axis(int i0, int i1, int n) {
  return (i0 == i1 && i1 == n - 1) ? n : i1;
}

// density_at for a binary16 volume from its quad copy q (grid qg, sizes nx+1, ny+1, nz): entry
// (a, b, k) holds the values at x corners a-1, a and y corners b-1, b (clamped) of plane k, so
// one 8-byte load per z plane gives four corners.  Same corners, weights and blend as
// density_at.
__device__ __forceinline__ float density_at_quad(const uint2 *__restrict__ q, const BrickGrid &qg,
                                                 const BrickGrid &g, f3 x) {
  if (!inside_cube(x)) return 0.0f;
  int i0, i1, j0, j1, k0, k1;
  float fx, fy, fz;
  tri_axis(x.x, g.nx, i0, i1, fx);
  tri_axis(x.y, g.ny, j0, j1, fy);
  tri_axis(x.z, g.nz, k0, k1, fz);
  const int oxy = brick_ox(quad_axis(i0, i1, g.nx)) + brick_oy(qg, quad_axis(j0, j1, g.ny));
  const uint2 p0 = q[oxy + brick_oz(qg, k0)], p1 = q[oxy + brick_oz(qg, k1)];
  auto h = [](uint32_t v) { return __half2float(__ushort_as_half((unsigned short)v)); };
  return trilerp8(h(p0.x & 0xFFFFu), h(p0.x >> 16), h(p0.y & 0xFFFFu), h(p0.y >> 16),
                  h(p1.x & 0xFFFFu), h(p1.x >> 16), h(p1.y & 0xFFFFu), h(p1.y >> 16), fx, fy, fz);
}

// The march kernels' density lookup: the quad copy when the volume has one.
template <typename T>
__device__ __forceinline__ float density_march(const T *__restrict__ vol, const BrickGrid &g,
                                               const uint2 *__restrict__ q, const BrickGrid &qg,
                                               f3 x) {
  if constexpr (sizeof(T) == 2) {
    if (q) return density_at_quad(q, qg, g, x);
  }
  return density_at(vol, g, x);
}

// Transfer function: 256 RGBA entries (float4) at density e/255, linear interpolation.
__device__ __forceinline__ float4 tf_lookup(const float4 *tf, float rho) {
  float u = fminf(fmaxf(rho * 255.0f, 0.0f), 255.0f);
  int i = min((int)floorf(u), 254);
  float f = u - (float)i;
  float4 a = tf[i], b = tf[i + 1];
  float g = 1.0f - f;
  return make_float4(g * a.x + f * b.x, g * a.y + f * b.y, g * a.z + f * b.z, g * a.w + f * b.w);
}

// ------------------------------------------------------------------ wave helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }
