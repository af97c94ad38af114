// Device helpers shared by the WCSPH and PCISPH kernels: block keys, the
// structural float operations, the cubic spline shape, wave reductions.
#pragma once

#include "rts_internal.h"

namespace rts {

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------
__device__ inline int clamp_cell(float f, int n) {
  if (!(f >= 0.0f)) return 0;  // negative or NaN
  if (f >= (float)(n - 1)) return n - 1;
  return (int)f;
}

// Block coordinates: t = x - o ; u = t * inv_e ; floor ; clamp.
__device__ inline int3 block_of(const DevParams &p, float x, float y, float z) {
#pragma clang fp contract(off)
  float tx = x - p.o[0], ty = y - p.o[1], tz = z - p.o[2];
  float ux = tx * p.inv_e, uy = ty * p.inv_e, uz = tz * p.inv_e;
  return make_int3(clamp_cell(floorf(ux), p.nc[0]), clamp_cell(floorf(uy), p.nc[1]),
                   clamp_cell(floorf(uz), p.nc[2]));
}
__device__ inline uint32_t key_of(const DevParams &p, int3 b) {
  return (uint32_t)(b.x + p.nc[0] * (b.y + p.nc[1] * b.z));
}
__device__ inline int3 coords_of(const DevParams &p, uint32_t k) {
  int bx = (int)(k % (uint32_t)p.nc[0]);
  uint32_t t = k / (uint32_t)p.nc[0];
  int by = (int)(t % (uint32_t)p.nc[1]);
  int bz = (int)(t / (uint32_t)p.nc[1]);
  return make_int3(bx, by, bz);
}

// |v|^2 = (vx*vx + vy*vy) + vz*vz, unfused.
__device__ inline float norm2_exact(float x, float y, float z) {
#pragma clang fp contract(off)
  float xx = x * x, yy = y * y, zz = z * z;
  float s = xx + yy;
  return s + zz;
}

// Squared distance from xj - xi per axis, as fma(dz, dz, fma(dy, dy, dx*dx)):
// each fused step is rounded once, so the CPU reproduces it with fmaf.
__device__ inline float dist2_exact(float xi, float yi, float zi, float xj, float yj, float zj) {
#pragma clang fp contract(off)
  const float dx = xj - xi, dy = yj - yi, dz = zj - zi;
  const float xx = dx * dx;
  return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, xx));
}

// Cubic spline shape w(q) and its derivative (support q < 2), branch-free:
// both pieces are evaluated and the right one selected.
__device__ inline float w_shape(float q) {
  const float w1 = 1.0f + q * q * (-1.5f + 0.75f * q);
  const float t = fmaxf(2.0f - q, 0.0f);
  const float w2 = 0.25f * t * t * t;
  return q < 1.0f ? w1 : w2;
}
__device__ inline float dw_shape(float q) {
  const float d1 = q * (-3.0f + 2.25f * q);
  const float t = fmaxf(2.0f - q, 0.0f);
  const float d2 = -0.75f * t * t;
  return q < 1.0f ? d1 : d2;
}

// Tait pressure from the density deviation d = rho/rho0 - 1, with
// (1 + d)^7 - 1 expanded in d (gamma = 7) so that nothing cancels.
__device__ inline float tait_from_dev(const DevParams &p, float d) {
  float poly = 7.0f + d * (21.0f + d * (35.0f + d * (35.0f + d * (21.0f + d * (7.0f + d)))));
  float pr = p.B * d * poly;
  if (p.clamp_p && pr < 0.0f) pr = 0.0f;
  return pr;
}

__device__ inline void set_status(DevScalars *S, uint32_t code, int32_t idx) {
  if (atomicCAS(&S->status, 0u, code) == 0u) S->bad_index = idx;
}

__device__ inline float wave_max(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline uint32_t wave_min_u32(uint32_t v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o, 64));
  return v;
}
__device__ inline uint32_t wave_sum_u32(uint32_t v) {
  for (int o = 32; o > 0; o >>= 1) v += (uint32_t)__shfl_xor((int)v, o, 64);
  return v;
}
__device__ inline uint32_t wave_max_u32(uint32_t v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, 64));
  return v;
}

}  // namespace rts
