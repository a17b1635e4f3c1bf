// Scene volumes on the device: the density volume in 8^3-brick order, its quad and cube copies
// (binary16 volumes: a cell's four (x, y) corners per z plane, or its eight corners, in one
// entry), and the light-transmittance grid (one f16 channel per light, half the volume
// resolution per axis).
#include "pfn_ctx.h"

template <typename T>
__global__ void brick_kernel(const T *__restrict__ src, T *__restrict__ dst, BrickGrid g) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t n = (size_t)g.nx * g.ny * g.nz;
  if (i >= n) return;
  int x = (int)(i % g.nx);
  int y = (int)((i / g.nx) % g.ny);
  int z = (int)(i / ((size_t)g.nx * g.ny));
  dst[brick_ox(x) + brick_oy(g, y) + brick_oz(g, z)] = src[i];
}

hipError_t launch_brick_volume(pfn_context *ctx, const void *src, pfn_dtype dt, int nx, int ny,
                               int nz) {
  size_t n = (size_t)nx * ny * nz;
  unsigned blocks = (unsigned)((n + 255) / 256);
  if (dt == PFN_F16)
    hipLaunchKernelGGL(brick_kernel<__half>, dim3(blocks), dim3(256), 0, ctx->stream,
                       (const __half *)src, (__half *)ctx->vol, ctx->vol_grid);
  else
    hipLaunchKernelGGL(brick_kernel<float>, dim3(blocks), dim3(256), 0, ctx->stream,
                       (const float *)src, (float *)ctx->vol, ctx->vol_grid);
  return hipGetLastError();
}

// Quad copy of a binary16 volume: entry (a, b, k) of grid qg (sizes nx+1, ny+1, nz) holds the
// values at (a-1, b-1), (a, b-1), (a-1, b), (a, b) of plane k, indices clamped to the volume.
__global__ void quad_kernel(const unsigned short *__restrict__ vol, BrickGrid vg,
                            uint2 *__restrict__ q, BrickGrid qg) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t n = (size_t)qg.nx * qg.ny * qg.nz;
  if (i >= n) return;
  const int a = (int)(i % qg.nx);
  const int b = (int)((i / qg.nx) % qg.ny);
  const int k = (int)(i / ((size_t)qg.nx * qg.ny));
  const int x0 = max(a - 1, 0), x1 = min(a, vg.nx - 1);
  const int y0 = max(b - 1, 0), y1 = min(b, vg.ny - 1);
  const int oz = brick_oz(vg, k);
  auto v = [&](int x, int y) { return (uint32_t)vol[brick_ox(x) + brick_oy(vg, y) + oz]; };
  q[brick_ox(a) + brick_oy(qg, b) + brick_oz(qg, k)] =
      make_uint2(v(x0, y0) | (v(x1, y0) << 16), v(x0, y1) | (v(x1, y1) << 16));
}

// Cube copy of a binary16 volume: entry (a, b, c) of grid cg (sizes nx+1, ny+1, nz+1) holds the
// values at x corners a-1, a, y corners b-1, b and z corners c-1, c (indices clamped to the
// volume), x fastest, so that one 16-byte load gives a trilinear lookup's eight corners.
__global__ void cube_kernel(const unsigned short *__restrict__ vol, BrickGrid vg,
                            uint4 *__restrict__ q, BrickGrid cg) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t n = (size_t)cg.nx * cg.ny * cg.nz;
  if (i >= n) return;
  const int a = (int)(i % cg.nx);
  const int b = (int)((i / cg.nx) % cg.ny);
  const int c = (int)(i / ((size_t)cg.nx * cg.ny));
  const int x0 = max(a - 1, 0), x1 = min(a, vg.nx - 1);
  const int y0 = max(b - 1, 0), y1 = min(b, vg.ny - 1);
  const int z0 = max(c - 1, 0), z1 = min(c, vg.nz - 1);
  auto v = [&](int x, int y, int z) {
    return (uint32_t)vol[brick_ox(x) + brick_oy(vg, y) + brick_oz(vg, z)];
  };
  q[brick_ox(a) + brick_oy(cg, b) + brick_oz(cg, c)] =
      make_uint4(v(x0, y0, z0) | (v(x1, y0, z0) << 16), v(x0, y1, z0) | (v(x1, y1, z0) << 16),
                 v(x0, y0, z1) | (v(x1, y0, z1) << 16), v(x0, y1, z1) | (v(x1, y1, z1) << 16));
}

hipError_t launch_cube_volume(pfn_context *ctx) {
  const BrickGrid &cg = ctx->cvol_grid;
  const size_t n = (size_t)cg.nx * cg.ny * cg.nz;  // below 2^31 (set_volume's bound)
  hipLaunchKernelGGL(cube_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ctx->stream,
                     (const unsigned short *)ctx->vol, ctx->vol_grid, ctx->cvol, cg);
  return hipGetLastError();
}

hipError_t launch_quad_volume(pfn_context *ctx) {
  const BrickGrid &qg = ctx->qvol_grid;
  size_t n = (size_t)qg.nx * qg.ny * qg.nz;
  hipLaunchKernelGGL(quad_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ctx->stream,
                     (const unsigned short *)ctx->vol, ctx->vol_grid, ctx->qvol, qg);
  return hipGetLastError();
}

struct LightVolArgs {
  const void *vol;
  const uint4 *cvol;  // cube copy of a binary16 volume, or NULL
  BrickGrid vg, cg, lvg;
  const float4 *tf;
  float ext_scale, step;
  int n_lights;
  float lp[4][3];
  ushort4 *out;
};

// exp(-17.5) = 2.5e-8 is below half the smallest binary16 subnormal (2^-25 = 3.0e-8): a
// transmittance at larger optical depth rounds to 0
#define LV_TAU_ZERO 17.5f

// Density of a binary16 volume from its cube copy at voxel coordinates u = x n - 0.5 (the
// cell-centre convention of tri_axis), with the corners, weights and blend of density_at: one
// 16-byte load.  The march's samples lie inside the cube; one that lands a rounding error
// outside takes the edge values, as the point inside does.  The y brick stride is below 2^24
// (at most 513 bricks of 512 entries), so its product runs at full rate; the z stride may
// exceed 2^24.
__device__ __forceinline__ float lv_density_cube(const uint4 *__restrict__ q, const BrickGrid &cg,
                                                 int nx, int ny, int nz, float ux, float uy,
                                                 float uz) {
  const float flx = floorf(ux), fly = floorf(uy), flz = floorf(uz);
  const float fx = ux - flx, fy = uy - fly, fz = uz - flz;
  const int lx = (int)flx, ly = (int)fly, lz = (int)flz;
  // cube entry (a, b, c): corners a-1, a / b-1, b / c-1, c, clamped (quad_axis of tri_axis)
  const int qa = min(max(lx + 1, 0), nx), qb = min(max(ly + 1, 0), ny),
            qc = min(max(lz + 1, 0), nz);
  const uint32_t o = (uint32_t)(((qa >> 3) << 9) + (qa & 7)) +
                     __umul24((uint32_t)(qb >> 3), (uint32_t)cg.sy) + (uint32_t)((qb & 7) << 3) +
                     (uint32_t)(qc >> 3) * (uint32_t)cg.sz + (uint32_t)((qc & 7) << 6);
  const uint4 p = q[o];
  auto h = [](uint32_t v) { return __half2float(__ushort_as_half((unsigned short)v)); };
  return trilerp8(h(p.x & 0xFFFFu), h(p.x >> 16), h(p.y & 0xFFFFu), h(p.y >> 16),
                  h(p.z & 0xFFFFu), h(p.z >> 16), h(p.w & 0xFFFFu), h(p.w >> 16), fx, fy, fz);
}

// U: march steps per pass of the cube-copy path (their density loads are in flight together)
template <typename VT, int U>
__global__ __launch_bounds__(256) void light_volume_kernel(LightVolArgs a) {
  __shared__ float4 tf[256];
  for (int i = threadIdx.x; i < 256; i += blockDim.x) tf[i] = a.tf[i];
  __syncthreads();
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t n = (size_t)a.lvg.nx * a.lvg.ny * a.lvg.nz;
  if (i >= n) return;
  int gx = (int)(i % a.lvg.nx);
  int gy = (int)((i / a.lvg.nx) % a.lvg.ny);
  int gz = (int)(i / ((size_t)a.lvg.nx * a.lvg.ny));
  f3 x = {((float)gx + 0.5f) / (float)a.lvg.nx, ((float)gy + 0.5f) / (float)a.lvg.ny,
          ((float)gz + 0.5f) / (float)a.lvg.nz};
  float T[4] = {1.f, 1.f, 1.f, 1.f};
  for (int l = 0; l < a.n_lights; ++l) {
    f3 p = {a.lp[l][0], a.lp[l][1], a.lp[l][2]};
    f3 v = p - x;
    float dist = sqrtf(dot(v, v));
    if (!(dist > 0.0f)) continue;
    f3 d = v * (1.0f / dist);
    float t0, t1;
    if (!clip_cube(x, d, t0, t1)) continue;
    float tend = fminf(t1, dist);
    if (!(tend > t0)) continue;
    float len = tend - t0, tau = 0.0f;
    // tau only grows (non-negative terms); past LV_TAU_ZERO the binary16 result is 0 whatever
    // the rest of the march adds, so the march stops there with the same output
    if (sizeof(VT) == 2 && a.cvol) {
      // binary16 volume: sample positions straight in voxel units, u = (x n - 0.5) + (d n) t
      const float nx = (float)a.vg.nx, ny = (float)a.vg.ny, nz = (float)a.vg.nz;
      const f3 u0 = {fmaf(x.x, nx, -0.5f), fmaf(x.y, ny, -0.5f), fmaf(x.z, nz, -0.5f)};
      const f3 du = {d.x * nx, d.y * ny, d.z * nz};
      // U steps per pass: their density loads are in flight together (each lookup clamps its
      // indices, so the steps past the end read valid entries and add nothing); the terms are
      // added in step order, and the stop test every U-th step gives the same output
      for (float kf = 0.0f; tau <= LV_TAU_ZERO; kf += (float)U) {
        float l_[U], rho[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
          const float kj = kf + (float)j;
          l_[j] = fminf(a.step, fmaf(-kj, a.step, len));
          const float t = fmaf(kj, a.step, fmaf(0.5f, l_[j], t0));
          rho[j] = lv_density_cube(a.cvol, a.cg, a.vg.nx, a.vg.ny, a.vg.nz, fmaf(du.x, t, u0.x),
                                   fmaf(du.y, t, u0.y), fmaf(du.z, t, u0.z));
        }
#pragma unroll
        for (int j = 0; j < U; ++j)
          if (l_[j] > 0.0f) tau = fmaf(tf_lookup(tf, rho[j]).w * a.ext_scale, l_[j], tau);
        if (!(l_[U - 1] > 0.0f)) break;
      }
    } else {
      for (int k = 0; tau <= LV_TAU_ZERO; ++k) {
        float l_ = fminf(a.step, len - (float)k * a.step);
        if (!(l_ > 0.0f)) break;
        float t = t0 + (float)k * a.step + 0.5f * l_;
        float rho = density_at(reinterpret_cast<const VT *>(a.vol), a.vg, x + d * t);
        tau = fmaf(tf_lookup(tf, rho).w * a.ext_scale, l_, tau);
      }
    }
    T[l] = expf(-tau);
  }
  ushort4 o;
  o.x = __half_as_ushort(__float2half_rn(T[0]));
  o.y = __half_as_ushort(__float2half_rn(T[1]));
  o.z = __half_as_ushort(__float2half_rn(T[2]));
  o.w = __half_as_ushort(__float2half_rn(T[3]));
  a.out[brick_ox(gx) + brick_oy(a.lvg, gy) + brick_oz(a.lvg, gz)] = o;
}

hipError_t launch_light_volume(pfn_context *ctx, float step) {
  LightVolArgs a{};
  a.vol = ctx->vol;
  a.cvol = ctx->vol_dtype == PFN_F16 && ctx->cvol_valid ? ctx->cvol : nullptr;
  a.vg = ctx->vol_grid;
  a.cg = ctx->cvol_grid;
  a.lvg = ctx->lv_grid;
  a.tf = ctx->tf_dev;
  a.ext_scale = ctx->ext_scale;
  a.step = step;
  a.n_lights = ctx->n_lights;
  for (int l = 0; l < ctx->n_lights; ++l)
    for (int c = 0; c < 3; ++c) a.lp[l][c] = ctx->lights[l].pos[c];
  a.out = ctx->lightvol;
  size_t n = (size_t)a.lvg.nx * a.lvg.ny * a.lvg.nz;
  unsigned blocks = (unsigned)((n + 255) / 256);
  // measured on 512^3 and 1024^3 binary16 volumes with 3 lights (bit-identical grids):
  //   quad copy (two 8-byte loads per lookup), 8 steps per pass: 63 ms / 1.58 s; 16 steps
  //   (230 registers, 2 waves per SIMD): 84 ms / 1.36 s;
  //   cube copy, 8 steps per pass (123 registers, 4 waves): 56.5 ms / 1.10 s; 16 steps: 72 ms /
  //   1.15 s.
  // A step's arithmetic (position, cell, blend, transfer function: about 60 vector
  // instructions) weighs more than its loads, so the one-load lookup gains 10-20 %.  The frame's
  // march kernels keep the quad copy: with the cube copy (twice its footprint) the 1080p field
  // frame took 28.5 against 27.95 ms and the cache-gather frame 6.5 against 6.35 ms.
  if (a.cvol)
    hipLaunchKernelGGL((light_volume_kernel<__half, 8>), dim3(blocks), dim3(256), 0, ctx->stream,
                       a);
  else if (ctx->vol_dtype == PFN_F16)
    hipLaunchKernelGGL((light_volume_kernel<__half, 1>), dim3(blocks), dim3(256), 0, ctx->stream,
                       a);
  else
    hipLaunchKernelGGL((light_volume_kernel<float, 1>), dim3(blocks), dim3(256), 0, ctx->stream,
                       a);
  return hipGetLastError();
}

// The light grid in plain x-fastest order (4 binary16 values per texel).
__global__ void light_unbrick_kernel(const ushort4 *__restrict__ lv, BrickGrid g,
                                     ushort4 *__restrict__ out) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t n = (size_t)g.nx * g.ny * g.nz;
  if (i >= n) return;
  const int x = (int)(i % g.nx);
  const int y = (int)((i / g.nx) % g.ny);
  const int z = (int)(i / ((size_t)g.nx * g.ny));
  out[i] = lv[brick_ox(x) + brick_oy(g, y) + brick_oz(g, z)];
}

hipError_t launch_light_unbrick(pfn_context *ctx, void *out) {
  const BrickGrid &g = ctx->lv_grid;
  size_t n = (size_t)g.nx * g.ny * g.nz;
  hipLaunchKernelGGL(light_unbrick_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     ctx->stream, ctx->lightvol, g, reinterpret_cast<ushort4 *>(out));
  return hipGetLastError();
}

// Quad copy of the light volume for up to 3 lights: entry (a, b, k) of grid qg (sizes nx+1,
// ny+1, nz of the light grid) holds channels 0-2 of the texels at (a-1, b-1), (a, b-1),
// (a-1, b), (a, b) of plane k (indices clamped), 12 binary16 values in 6 dwords.
__global__ void light_quad_kernel(const ushort4 *__restrict__ lv, BrickGrid g,
                                  uint32_t *__restrict__ q, BrickGrid qg) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t n = (size_t)qg.nx * qg.ny * qg.nz;
  if (i >= n) return;
  const int a = (int)(i % qg.nx);
  const int b = (int)((i / qg.nx) % qg.ny);
  const int k = (int)(i / ((size_t)qg.nx * qg.ny));
  const int x0 = max(a - 1, 0), x1 = min(a, g.nx - 1);
  const int y0 = max(b - 1, 0), y1 = min(b, g.ny - 1);
  const int oz = brick_oz(g, k);
  const ushort4 t00 = lv[brick_ox(x0) + brick_oy(g, y0) + oz];
  const ushort4 t10 = lv[brick_ox(x1) + brick_oy(g, y0) + oz];
  const ushort4 t01 = lv[brick_ox(x0) + brick_oy(g, y1) + oz];
  const ushort4 t11 = lv[brick_ox(x1) + brick_oy(g, y1) + oz];
  uint32_t *o = q + 6 * (size_t)(brick_ox(a) + brick_oy(qg, b) + brick_oz(qg, k));
  auto w = [](unsigned short lo, unsigned short hi) { return (uint32_t)lo | ((uint32_t)hi << 16); };
  o[0] = w(t00.x, t00.y);
  o[1] = w(t00.z, t10.x);
  o[2] = w(t10.y, t10.z);
  o[3] = w(t01.x, t01.y);
  o[4] = w(t01.z, t11.x);
  o[5] = w(t11.y, t11.z);
}

hipError_t launch_light_quad(pfn_context *ctx) {
  const BrickGrid &qg = ctx->lquad_grid;
  size_t n = (size_t)qg.nx * qg.ny * qg.nz;
  hipLaunchKernelGGL(light_quad_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     ctx->stream, ctx->lightvol, ctx->lv_grid, ctx->lquad, qg);
  return hipGetLastError();
}
