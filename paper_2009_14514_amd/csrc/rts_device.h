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

// Combines two Kahan accumulators (true value = s - c), the rounding of the
// sum s + s2 being carried into c.
__device__ inline void kahan_merge(float &s, float &c, float s2, float c2) {
  const float t = s + s2;
  const float v = t - s;
  const float e = (s - (t - v)) + (s2 - v);  // t + e == s + s2 exactly
  s = t;
  c = (c + c2) - e;
}

// ---------------------------------------------------------------------------
// a block's 27-block candidate set, staged in LDS (search, force, the lists
// of the differentiable substep)
// ---------------------------------------------------------------------------
constexpr int kStageCap = 2048;               // candidates staged in LDS (search: 16 B each)
constexpr int kForceCap = 2048;               // candidates staged in LDS (force: 32 B each)

// The candidate set of a block: 9 fluid row ranges (dz outer, dy inner, each
// row covering x-1..x+1 contiguously in sorted order) followed by the same 9
// rows of the wall grid.  Range r starts at global index rs and occupies
// local indices [ro[r], ro[r+1]).  Local order equals the canonical
// neighbour order (ascending sorted index, fluid before walls).
__device__ inline void row_range(const DevParams &p, const uint32_t *start,
                                 const uint32_t *wstart, int3 c, int r, uint32_t &rs,
                                 uint32_t &len) {
  const uint32_t *cs = r < 9 ? start : wstart;
  const int rr = r % 9;
  const int z = c.z + rr / 3 - 1, y = c.y + rr % 3 - 1;
  rs = 0;
  len = 0;
  if (z < 0 || z >= p.nc[2] || y < 0 || y >= p.nc[1]) return;
  if (r >= 9 && p.nw == 0) return;
  const int x0 = max(c.x - 1, 0), x1 = min(c.x + 1, p.nc[0] - 1);
  const uint32_t row = (uint32_t)p.nc[0] * ((uint32_t)y + (uint32_t)p.nc[1] * (uint32_t)z);
  rs = cs[row + (uint32_t)x0];
  const uint32_t re = cs[row + (uint32_t)x1 + 1u];
  len = re > rs ? re - rs : 0u;
}

// Global position of local candidate k.
__device__ inline uint32_t local_to_global(const uint32_t *rs, const uint32_t *ro, uint32_t k,
                                           bool &wall) {
  int r = 0;
  while (r < 17 && k >= ro[r + 1]) ++r;
  wall = r >= 9;
  return rs[r] + (k - ro[r]);
}

// Position of candidate k (< C) for staging; j = its fluid index, or kNoFluid
// for a wall particle or a slot past the candidates.
constexpr uint32_t kNoFluid = 0xFFFFFFFFu;
__device__ inline float4 stage_load(const uint32_t *rs, const uint32_t *ro,
                                    const float4 *__restrict__ P, const float4 *__restrict__ WP,
                                    uint32_t k, uint32_t C, uint32_t &j) {
  j = kNoFluid;
  if (k >= C) return make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  bool wall;
  const uint32_t g = local_to_global(rs, ro, k, wall);
  if (!wall) j = g;
  return wall ? WP[g] : P[g];
}

// Sets up the candidate ranges of block b in shared memory and their prefix
// offsets.  Ends with the offsets visible to the whole workgroup.
__device__ inline void block_ranges_shared(const DevParams &p, const uint32_t *start,
                                           const uint32_t *wstart, uint32_t b, uint32_t *s_rs,
                                           uint32_t *s_ro, uint32_t *s_len) {
  const int tid = threadIdx.x;
  if (tid < 64) {
    // one wave: the 18 lengths and their exclusive prefix by shuffles
    uint32_t rs = 0, len = 0;
    if (tid < 18) row_range(p, start, wstart, coords_of(p, b), tid, rs, len);
    uint32_t v = len;
#pragma unroll
    for (int o = 1; o < 32; o <<= 1) {
      const uint32_t u = (uint32_t)__shfl_up((int)v, o, 64);
      if ((tid & 63) >= o) v += u;
    }
    if (tid < 18) {
      s_rs[tid] = rs;
      s_len[tid] = len;
      s_ro[tid] = v - len;
    }
    if (tid == 17) s_ro[18] = v;
  }
  __syncthreads();
}

// A staged position without the fourth component (12 bytes in LDS).
struct Pos3 {
  float x, y, z;
};
__device__ inline void put_pos(float4 *s, uint32_t k, const float4 v) { s[k] = v; }
__device__ inline void put_pos(Pos3 *s, uint32_t k, const float4 v) { s[k] = Pos3{v.x, v.y, v.z}; }

// Copies the block's candidates into shared memory in canonical order, one
// range at a time so that consecutive threads read consecutive particles;
// slots from C up to cpad are filled with far-away positions.
template <int kThreads, typename Slot>
__device__ inline void stage_positions(const uint32_t *s_rs, const uint32_t *s_ro,
                                       const float4 *__restrict__ P,
                                       const float4 *__restrict__ WP, Slot *s_pos,
                                       uint32_t cpad) {
  constexpr int kPer = (kStageCap + kThreads - 1) / kThreads;
  const uint32_t C = s_ro[18];
  float4 v[kPer];
  // every load is issued before the first shared-memory write
#pragma unroll
  for (int it = 0; it < kPer; ++it) {
    const uint32_t k = (uint32_t)threadIdx.x + (uint32_t)it * kThreads;
    v[it] = make_float4(1e30f, 1e30f, 1e30f, 0.0f);  // padding: never a neighbour
    if (k < C) {
      bool wall;
      const uint32_t j = local_to_global(s_rs, s_ro, k, wall);
      v[it] = wall ? WP[j] : P[j];
    }
  }
#pragma unroll
  for (int it = 0; it < kPer; ++it) {
    const uint32_t k = (uint32_t)threadIdx.x + (uint32_t)it * kThreads;
    if (k < cpad) put_pos(s_pos, k, v[it]);
  }
}

}  // namespace rts
