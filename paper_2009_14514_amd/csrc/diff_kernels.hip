// HIP kernels of the differentiable WCSPH substep and its adjoint on gfx950.
//
// Forward substep (every particle active, symplectic Euler), particles in the
// caller's order:
//   rho_i = m (W(0) + sum_j W_ij + sum_w W_iw),  p_i = B ((rho_i/rho0)^7 - 1)
//   a_i   = g - sum_j m (P_i + P_j + Pi_ij) gradW_ij - sum_w m (2 P_i + Pi_iw) gradW_iw
//   v' = v + dt a,  x' = x + dt v'
// with P = p / rho^2 and the Monaghan viscosity Pi (approaching pairs only).
//
// The adjoint is in gather form: particle i visits its own list once and
// collects its share of every pair's partial derivatives, using that the
// neighbour relation is symmetric and that a pair enters a_i and a_j with
// opposite signs, so the pair's upstream gradient is abar_j - abar_i.  No
// thread writes another particle's adjoint, so no atomics are needed.  Lists
// are built per block from LDS-staged candidates.  The pair sums give a
// particle kDiffSub lanes (lane s takes list entries s, s + kDiffSub, ...),
// whose partial sums are folded in a fixed order: runs are deterministic.
#include "rts_device.h"
#include "xcd.h"

namespace rts {

// lanes per particle in the pair sums: one lane per particle leaves too few
// waves to hide the gathers' latency at 100k particles
constexpr int kDiffSub = 8;

// the lanes of a particle: its index and this lane's rank among them
__device__ inline int diff_particle(int &s) {
  const uint32_t t = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  s = (int)(t % (uint32_t)kDiffSub);
  return (int)(t / (uint32_t)kDiffSub);
}
// fixed-order fold of the kDiffSub lanes' partial sums
__device__ inline float diff_fold(float v) {
  for (int o = 1; o < kDiffSub; o <<= 1) v += __shfl_xor(v, o, kDiffSub);
  return v;
}

struct DiffArgs {
  float dt, B, alpha, hc0;  // step, Tait stiffness, viscosity alpha, h c0
  int32_t n, cap;           // particles, list entries per particle
};

__device__ inline float d2w_shape(float q) {
  const float a = -3.0f + 4.5f * q;
  const float b = 1.5f * fmaxf(2.0f - q, 0.0f);
  return q < 1.0f ? a : b;
}

// (1 + d)^7 - 1 and its derivative 7 (1 + d)^6, expanded in d
__device__ inline float pow7m1(float d) {
  return d * (7.0f + d * (21.0f + d * (35.0f + d * (35.0f + d * (21.0f + d * (7.0f + d))))));
}
__device__ inline float pow6(float d) {
  const float t = 1.0f + d;
  const float t3 = t * t * t;
  return t3 * t3;
}

__global__ void k_diff_copy_in(DiffArgs a, const float4 *__restrict__ X, float4 *__restrict__ P,
                               float4 *__restrict__ V, float4 *__restrict__ A,
                               uint32_t *__restrict__ M, uint32_t *__restrict__ ID) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const float4 x = X[i];
  P[i] = make_float4(x.x, x.y, x.z, 0.0f);
  V[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  A[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  M[i] = 0u;
  ID[i] = (uint32_t)i;
}

// Lists in the canonical order of the sorted grid (rows dz, dy; blocks in x),
// entries are caller indices (fluid) or wall sorted index | bit 31.
//
// One workgroup per occupied block: the block's 27-block candidate set is
// staged in LDS in canonical order together with each candidate's list entry
// (caller index, or wall sorted index | bit 31); kSub lanes share a particle
// and test interleaved candidates, and a ballot of the group's hits over each
// run of kSub consecutive candidates places them in the canonical order.  A
// block with more candidates than LDS slots is scanned from memory by one
// lane per particle.  Lists are particle-major (entry k of particle i at
// i * cap + k): a ballot's hits land in consecutive words, and the pair
// passes' lanes of a particle read consecutive words.
constexpr int kDiffListThreads = 512;
__global__ void __launch_bounds__(kDiffListThreads) k_diff_lists_blocks(
    DevParams p, DiffArgs a, const float4 *__restrict__ Ps, const uint32_t *__restrict__ perm,
    const uint32_t *__restrict__ occ, const uint32_t *__restrict__ start,
    const float4 *__restrict__ WP, const uint32_t *__restrict__ wstart, uint32_t *__restrict__ L,
    uint32_t *__restrict__ nn, DevScalars *S) {
  __shared__ float4 s_pos[kStageCap];
  __shared__ uint32_t s_code[kStageCap];
  __shared__ uint32_t s_rs[18], s_ro[19], s_len[18];
  const uint32_t tid = threadIdx.x;
  const uint32_t sub = tid & (uint32_t)(kSub - 1);
  const uint32_t first = (tid & 63u) & ~(uint32_t)(kSub - 1);  // the group's first lane
  const uint32_t wave_first_slot = (tid / 64u) * (64u / kSub);
  const uint32_t nocc = S->n_occ;
  for (uint32_t q = xcd_block(blockIdx.x, gridDim.x); q < nocc; q += gridDim.x) {
    const uint32_t b = occ[q];
    const uint32_t s0 = start[b];
    const uint32_t nb = start[b + 1] - s0;
    block_ranges_shared(p, start, wstart, b, s_rs, s_ro, s_len);
    const uint32_t C = s_ro[18];
    const uint32_t cpad = (C + kSub - 1) / kSub * kSub;
    const bool staged = cpad <= (uint32_t)kStageCap;
    if (staged)
      for (uint32_t k = tid; k < cpad; k += kDiffListThreads) {
        float4 v = make_float4(1e30f, 1e30f, 1e30f, 0.0f);  // padding: never a neighbour
        uint32_t code = 0u;
        if (k < C) {
          bool wall;
          const uint32_t g = local_to_global(s_rs, s_ro, k, wall);
          v = wall ? WP[g] : Ps[g];
          code = wall ? (g | kWallBit) : perm[g];
        }
        s_pos[k] = v;
        s_code[k] = code;
      }
    __syncthreads();
    const uint32_t self_off = s_ro[4] - s_rs[4];  // local index = sorted index + self_off
    for (uint32_t c0 = 0; c0 < nb; c0 += kDiffListThreads / kSub) {
      if (c0 + wave_first_slot >= nb) break;  // no particle for this wave
      const uint32_t slot = c0 + tid / kSub;
      const bool live = slot < nb;
      const uint32_t s = s0 + (live ? slot : 0u);
      const uint32_t i = perm[s];  // caller index
      const float4 xi = Ps[s];
      uint32_t *out = L + (size_t)i * (size_t)a.cap;  // particle-major
      uint32_t cnt = 0;  // the same in the group's lanes
      if (staged) {
        const uint32_t selfk = s + self_off;
        for (uint32_t base = 0; base < cpad; base += kSub) {
          const uint32_t k = base + sub;
          const float4 qj = s_pos[k];
          const bool hit =
              live && k != selfk && dist2_exact(xi.x, xi.y, xi.z, qj.x, qj.y, qj.z) < p.r2f;
          const uint32_t mask = (uint32_t)(__ballot(hit) >> first) & ((1u << kSub) - 1u);
          if (hit) {
            const uint32_t pos = cnt + (uint32_t)__popc(mask & ((1u << sub) - 1u));
            if (pos < (uint32_t)a.cap) out[pos] = s_code[k];
          }
          cnt += (uint32_t)__popc(mask);
        }
      } else if (live && sub == 0u) {
        for (uint32_t k = 0; k < C; ++k) {
          bool wall;
          const uint32_t g = local_to_global(s_rs, s_ro, k, wall);
          if (!wall && g == s) continue;
          const float4 qj = wall ? WP[g] : Ps[g];
          if (!(dist2_exact(xi.x, xi.y, xi.z, qj.x, qj.y, qj.z) < p.r2f)) continue;
          if (cnt < (uint32_t)a.cap) out[cnt] = wall ? (g | kWallBit) : perm[g];
          ++cnt;
        }
      }
      if (live && sub == 0u) {
        if (cnt > (uint32_t)a.cap) {
          set_status(S, RTS_E_CAPACITY, (int32_t)i);
          cnt = (uint32_t)a.cap;
        }
        nn[i] = cnt;
      }
    }
    __syncthreads();  // shared memory is reused by the next block
  }
}

// Density by summation (compensated) and the unclamped Tait pressure, both
// from the deviation d = rho/rho0 - 1 formed before rounding to rho.  The
// force pass gathers two float4 per neighbour: (x, P) with P = p / rho^2 and
// (v, rho), packed here.
__global__ void __launch_bounds__(256) k_diff_density(
    DevParams p, DiffArgs a, const float4 *__restrict__ X, const float4 *__restrict__ V,
    const uint32_t *__restrict__ L, const uint32_t *__restrict__ nn,
    const float4 *__restrict__ WP, float *__restrict__ rho, float *__restrict__ prs,
    float4 *__restrict__ XP, float4 *__restrict__ VR) {
  int s;
  const int i = diff_particle(s);
  if (i >= a.n) return;  // the particle's lanes leave together
  const float4 xi = X[i];
  const uint32_t *row = L + (size_t)i * (size_t)a.cap;
  const uint32_t cnt = nn[i];
  float sum = 0.0f, comp = 0.0f;
#pragma unroll 4
  for (uint32_t k = (uint32_t)s; k < cnt; k += kDiffSub) {
    const uint32_t j = row[k];
    const float4 q = (j & kWallBit) ? WP[j & ~kWallBit] : X[j];
    const float dx = xi.x - q.x, dy = xi.y - q.y, dz = xi.z - q.z;
    const float w = w_shape(__builtin_sqrtf(dx * dx + dy * dy + dz * dz) * p.inv_h);
    const float y = w - comp;
    const float t = sum + y;
    comp = (t - sum) - y;
    sum = t;
  }
  for (int o = 1; o < kDiffSub; o <<= 1) {
    const float s2 = __shfl_xor(sum, o, kDiffSub), c2 = __shfl_xor(comp, o, kDiffSub);
    kahan_merge(sum, comp, s2, c2);
  }
  if (s != 0) return;
  const float dev = p.kms * ((sum - p.c_hi) - (comp + p.c_lo));
  const float r = p.rho0 + p.rho0 * dev, pr = a.B * pow7m1(dev);
  rho[i] = r;
  prs[i] = pr;
  const float4 vi = V[i];
  XP[i] = make_float4(xi.x, xi.y, xi.z, pr / (r * r));
  VR[i] = make_float4(vi.x, vi.y, vi.z, r);
}

__global__ void __launch_bounds__(256) k_diff_force_euler(
    DevParams p, DiffArgs a, const float4 *__restrict__ XP, const float4 *__restrict__ VR,
    const uint32_t *__restrict__ L, const uint32_t *__restrict__ nn,
    const float4 *__restrict__ WP, float4 *__restrict__ Xn, float4 *__restrict__ Vn) {
  int sl;
  const int i = diff_particle(sl);
  if (i >= a.n) return;  // the particle's lanes leave together
  const float4 xi = XP[i], vi = VR[i];
  const float ri = vi.w, Pi = xi.w;
  const float nu_wall = a.alpha * a.hc0 * __builtin_amdgcn_rcpf(ri);
  const uint32_t *row = L + (size_t)i * (size_t)a.cap;
  const uint32_t cnt = nn[i];
  float ax = 0.0f, ay = 0.0f, az = 0.0f;
#pragma unroll 4
  for (uint32_t k = (uint32_t)sl; k < cnt; k += kDiffSub) {
    const uint32_t j = row[k];
    const bool wall = (j & kWallBit) != 0u;
    float4 q, u = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float coef, nu;
    if (wall) {
      q = WP[j & ~kWallBit];
      coef = 2.0f * Pi;
      nu = nu_wall;
    } else {
      q = XP[j];
      u = VR[j];
      coef = Pi + q.w;
      nu = 2.0f * a.alpha * a.hc0 * __builtin_amdgcn_rcpf(ri + u.w);
    }
    const float dx = xi.x - q.x, dy = xi.y - q.y, dz = xi.z - q.z;
    const float r2 = dx * dx + dy * dy + dz * dz;
    if (!(r2 > 0.0f) || r2 >= p.r2f) continue;
    const float sv = (vi.x - u.x) * dx + (vi.y - u.y) * dy + (vi.z - u.z) * dz;
    if (sv < 0.0f) coef += -nu * sv * __builtin_amdgcn_rcpf(r2 + p.visc_eps_h2);
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float F = p.sigma * p.inv_h * dw_shape(r2 * rinv * p.inv_h) * rinv;
    const float t = p.mass * coef * F;
    ax -= t * dx;
    ay -= t * dy;
    az -= t * dz;
  }
  ax = p.g[0] + diff_fold(ax);
  ay = p.g[1] + diff_fold(ay);
  az = p.g[2] + diff_fold(az);
  if (sl != 0) return;
  const float vx = vi.x + a.dt * ax, vy = vi.y + a.dt * ay, vz = vi.z + a.dt * az;
  Vn[i] = make_float4(vx, vy, vz, 0.0f);
  Xn[i] = make_float4(xi.x + a.dt * vx, xi.y + a.dt * vy, xi.z + a.dt * vz, 0.0f);
}

// x' = x + dt v', v' = v + dt a: vbar <- vbar' + dt xbar', abar = dt vbar (xbar
// unchanged).  Also packs the frame as (x, rho) and (v, p) for the adjoint
// force pass, which then gathers two float4 per neighbour besides abar.
__global__ void k_diff_adj_euler(DiffArgs a, const float4 *__restrict__ XB, float4 *__restrict__ VB,
                                 float4 *__restrict__ AB, const float4 *__restrict__ X,
                                 const float4 *__restrict__ V, const float *__restrict__ rho,
                                 const float *__restrict__ prs, float4 *__restrict__ XR,
                                 float4 *__restrict__ VP) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const float4 x = X[i], v = V[i];
  XR[i] = make_float4(x.x, x.y, x.z, rho[i]);
  VP[i] = make_float4(v.x, v.y, v.z, prs[i]);
  const float4 xb = XB[i];
  float4 vb = VB[i];
  vb.x += a.dt * xb.x;
  vb.y += a.dt * xb.y;
  vb.z += a.dt * xb.z;
  VB[i] = vb;
  AB[i] = make_float4(a.dt * vb.x, a.dt * vb.y, a.dt * vb.z, 0.0f);
}

// Adjoint of the forces, the pressure p / rho^2 and the equation of state.
// The frame comes packed as (x, rho), (v, p); rbar leaves packed with x as
// (x, rbar) for the density adjoint.
__global__ void __launch_bounds__(256) k_diff_adj_force(
    DevParams p, DiffArgs a, const float4 *__restrict__ XR, const float4 *__restrict__ VP,
    const uint32_t *__restrict__ L, const uint32_t *__restrict__ nn,
    const float4 *__restrict__ WP, const float4 *__restrict__ AB, float4 *__restrict__ XB,
    float4 *__restrict__ VB, float4 *__restrict__ XRB, double *__restrict__ BB,
    double *__restrict__ AA) {
  int sl;
  const int i = diff_particle(sl);
  if (i >= a.n) return;  // the particle's lanes leave together
  const float4 xi = XR[i], vi = VP[i], abi = AB[i];
  const float ri = xi.w, pi = vi.w, Pi = pi / (ri * ri);
  const uint32_t *row = L + (size_t)i * (size_t)a.cap;
  const uint32_t cnt = nn[i];
  const float m = p.mass, e = p.visc_eps_h2;
  const float inv_h2 = p.inv_h * p.inv_h;
  // reciprocals from the hardware's rcp / rsq (about 1 ulp)
  const float iri = __builtin_amdgcn_rcpf(ri), inv_alpha = __builtin_amdgcn_rcpf(a.alpha);
  float gxx = 0.0f, gxy = 0.0f, gxz = 0.0f, gvx = 0.0f, gvy = 0.0f, gvz = 0.0f;
  float Pb = 0.0f, rb = 0.0f, alb = 0.0f;
#pragma unroll 4
  for (uint32_t k = (uint32_t)sl; k < cnt; k += kDiffSub) {
    const uint32_t j = row[k];
    const bool wall = (j & kWallBit) != 0u;
    float4 q, vj = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float coef, nu, isum = iri, ux, uy, uz;  // isum: 1 / (rho_i + rho_j), 1 / rho_i at a wall
    if (wall) {
      q = WP[j & ~kWallBit];
      coef = 2.0f * Pi;
      nu = a.alpha * a.hc0 * iri;
      ux = -abi.x;
      uy = -abi.y;
      uz = -abi.z;
    } else {
      q = XR[j];
      vj = VP[j];
      const float irj = __builtin_amdgcn_rcpf(q.w);
      coef = Pi + vj.w * irj * irj;
      isum = __builtin_amdgcn_rcpf(ri + q.w);
      nu = 2.0f * a.alpha * a.hc0 * isum;
      const float4 abj = AB[j];
      ux = abj.x - abi.x;
      uy = abj.y - abi.y;
      uz = abj.z - abi.z;
    }
    const float dx = xi.x - q.x, dy = xi.y - q.y, dz = xi.z - q.z;
    const float r2 = dx * dx + dy * dy + dz * dz;
    if (!(r2 > 0.0f) || r2 >= p.r2f) continue;
    const float rinv = __builtin_amdgcn_rsqf(r2), r = r2 * rinv;
    const float wx = vi.x - vj.x, wy = vi.y - vj.y, wz = vi.z - vj.z;
    const float s = wx * dx + wy * dy + wz * dz;
    const bool visc = s < 0.0f;
    const float iden = __builtin_amdgcn_rcpf(r2 + e);
    if (visc) coef += -nu * s * iden;
    const float qn = r * p.inv_h;
    const float W1 = p.sigma * p.inv_h * dw_shape(qn), W2 = p.sigma * inv_h2 * d2w_shape(qn);
    const float F = W1 * rinv, dF = (W2 * r - W1) * rinv * rinv;
    const float Gu = F * (dx * ux + dy * uy + dz * uz);
    const float xu = dx * ux + dy * uy + dz * uz;
    const float c1 = m * coef * F, c2 = m * coef * dF * rinv * xu;
    gxx += c1 * ux + c2 * dx;
    gxy += c1 * uy + c2 * dy;
    gxz += c1 * uz + c2 * dz;
    if (visc) {
      const float mg = m * Gu;
      const float k1 = -nu * iden, k2 = 2.0f * nu * s * iden * iden;
      gxx += (k1 * wx + k2 * dx) * mg;
      gxy += (k1 * wy + k2 * dy) * mg;
      gxz += (k1 * wz + k2 * dz) * mg;
      gvx += k1 * dx * mg;
      gvy += k1 * dy * mg;
      gvz += k1 * dz * mg;
      const float nub = -s * iden * mg;
      rb += nub * (-nu * isum);
      if (wall) {
        alb += nub * nu * inv_alpha;
      } else {
        alb += 0.5f * nub * nu * inv_alpha;   // the pair is visited from both ends
      }
    }
    Pb += (wall ? 2.0f : 1.0f) * m * Gu;
  }
  gxx = diff_fold(gxx);
  gxy = diff_fold(gxy);
  gxz = diff_fold(gxz);
  gvx = diff_fold(gvx);
  gvy = diff_fold(gvy);
  gvz = diff_fold(gvz);
  Pb = diff_fold(Pb);
  rb = diff_fold(rb);
  alb = diff_fold(alb);
  if (sl != 0) return;
  // P = p / rho^2 ; p = B ((1 + d)^7 - 1), d = rho / rho0 - 1
  const float dev = ri / p.rho0 - 1.0f;
  const float pb = Pb / (ri * ri);
  rb += Pb * (-2.0f * pi / (ri * ri * ri)) + pb * 7.0f * a.B * pow6(dev) / p.rho0;
  BB[i] += (double)pb * (double)pow7m1(dev);
  AA[i] += (double)alb;
  float4 xb = XB[i], vb = VB[i];
  xb.x += gxx;
  xb.y += gxy;
  xb.z += gxz;
  vb.x += gvx;
  vb.y += gvy;
  vb.z += gvz;
  XB[i] = xb;
  VB[i] = vb;
  XRB[i] = make_float4(xi.x, xi.y, xi.z, rb);
}

// Adjoint of the density summation: xbar_i += sum_j m gradW_ij (rbar_i + rbar_j).
__global__ void __launch_bounds__(256) k_diff_adj_density(
    DevParams p, DiffArgs a, const float4 *__restrict__ XRB, const uint32_t *__restrict__ L,
    const uint32_t *__restrict__ nn, const float4 *__restrict__ WP, float4 *__restrict__ XB) {
  int s;
  const int i = diff_particle(s);
  if (i >= a.n) return;  // the particle's lanes leave together
  const float4 xi = XRB[i];
  const float rbi = xi.w;
  const uint32_t *row = L + (size_t)i * (size_t)a.cap;
  const uint32_t cnt = nn[i];
  float gx = 0.0f, gy = 0.0f, gz = 0.0f;
#pragma unroll 4
  for (uint32_t k = (uint32_t)s; k < cnt; k += kDiffSub) {
    const uint32_t j = row[k];
    const bool wall = (j & kWallBit) != 0u;
    const float4 q = wall ? WP[j & ~kWallBit] : XRB[j];
    const float rs = wall ? rbi : rbi + q.w;
    const float dx = xi.x - q.x, dy = xi.y - q.y, dz = xi.z - q.z;
    const float r2 = dx * dx + dy * dy + dz * dz;
    if (!(r2 > 0.0f) || r2 >= p.r2f) continue;
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float t = p.mass * p.sigma * p.inv_h * dw_shape(r2 * rinv * p.inv_h) * rinv * rs;
    gx += t * dx;
    gy += t * dy;
    gz += t * dz;
  }
  gx = diff_fold(gx);
  gy = diff_fold(gy);
  gz = diff_fold(gz);
  if (s != 0) return;
  float4 xb = XB[i];
  xb.x += gx;
  xb.y += gy;
  xb.z += gz;
  XB[i] = xb;
}

// planes <-> float4
__global__ void k_diff_planes_in(int n, const float *__restrict__ src, float4 *__restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  dst[i] = make_float4(src[i], src[n + i], src[2 * n + i], 0.0f);
}
__global__ void k_diff_planes_out(int n, const float4 *__restrict__ src, float *__restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 v = src[i];
  dst[i] = v.x;
  dst[n + i] = v.y;
  dst[2 * n + i] = v.z;
}
__global__ void k_diff_zero(int n, float4 *__restrict__ a, double *__restrict__ b,
                            double *__restrict__ c) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (a) a[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  b[i] = 0.0;
  c[i] = 0.0;
}

// One workgroup: fixed-order sums of the two per-particle accumulators.
__global__ void __launch_bounds__(256) k_diff_reduce(int n, const double *__restrict__ BB,
                                                    const double *__restrict__ AA,
                                                    double *__restrict__ out) {
  __shared__ double s_b[256], s_a[256];
  const int t = threadIdx.x;
  double sb = 0.0, sa = 0.0;
  int i = t;
  // four entries' loads issued before they are added (in the same order)
  for (; i + 3 * 256 < n; i += 4 * 256) {
    const double b0 = BB[i], b1 = BB[i + 256], b2 = BB[i + 512], b3 = BB[i + 768];
    const double a0 = AA[i], a1 = AA[i + 256], a2 = AA[i + 512], a3 = AA[i + 768];
    sb += b0;
    sb += b1;
    sb += b2;
    sb += b3;
    sa += a0;
    sa += a1;
    sa += a2;
    sa += a3;
  }
  for (; i < n; i += 256) {
    sb += BB[i];
    sa += AA[i];
  }
  s_b[t] = sb;
  s_a[t] = sa;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) {
      s_b[t] += s_b[t + o];
      s_a[t] += s_a[t + o];
    }
    __syncthreads();
  }
  if (t == 0) {
    out[0] = s_b[0];
    out[1] = s_a[0];
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {
unsigned dgrid(int64_t n) { return (unsigned)(n > 0 ? (n + 255) / 256 : 1); }
DiffArgs dargs(int n, int cap, float dt, float B, float alpha, float hc0) {
  DiffArgs a;
  a.dt = dt;
  a.B = B;
  a.alpha = alpha;
  a.hc0 = hc0;
  a.n = n;
  a.cap = cap;
  return a;
}
}  // namespace

void launch_diff_planes_in(int n, const float *src, float4 *dst, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_diff_planes_in, dim3(dgrid(n)), dim3(256), 0, st, n, src, dst);
}
void launch_diff_planes_out(int n, const float4 *src, float *dst, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_diff_planes_out, dim3(dgrid(n)), dim3(256), 0, st, n, src, dst);
}
void launch_diff_zero(int n, float4 *a, double *b, double *c, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_diff_zero, dim3(dgrid(n)), dim3(256), 0, st, n, a, b, c);
}

// Lists, density and pressure of the state X (caller order): the sort of
// the WCSPH path supplies the canonical block order.
void launch_diff_setup(const DevParams &p, const DevPtrs &d, int n, int cap, float B,
                       const float4 *X, const float4 *V, uint32_t *L, uint32_t *nn, float *rho,
                       float *prs, float4 *XP, float4 *VR, int grid_wave, hipStream_t st) {
  const DiffArgs a = dargs(n, cap, 0.0f, B, 0.0f, 0.0f);
  if (n > 0)
    hipLaunchKernelGGL(k_diff_copy_in, dim3(dgrid(n)), dim3(256), 0, st, a, X, d.P[0], d.V[0],
                       d.A[0], d.M[0], d.ID[0]);
  launch_key_hist(p, d, 0, st);
  launch_scan(p, d, d.CELL_START, true, st);
  launch_scatter(p, d, st);
  launch_cell_gather(p, d, 0, grid_wave, st);
  if (n == 0) return;
  hipLaunchKernelGGL(k_diff_lists_blocks, dim3(1024), dim3(kDiffListThreads), 0, st, p, a,
                     d.P[1], d.PERM, d.OCC, d.CELL_START, d.WP, d.WCELL_START, L, nn, d.S);
  hipLaunchKernelGGL(k_diff_density, dim3(dgrid((int64_t)n * kDiffSub)), dim3(256), 0, st, p, a, X, V, L, nn, d.WP,
                     rho, prs, XP, VR);
}
void launch_diff_force_euler(const DevParams &p, const DevPtrs &d, int n, int cap, float dt,
                             float alpha, float hc0, const float4 *XP, const float4 *VR,
                             const uint32_t *L, const uint32_t *nn, float4 *Xn, float4 *Vn,
                             hipStream_t st) {
  if (n == 0) return;
  const DiffArgs a = dargs(n, cap, dt, 0.0f, alpha, hc0);
  hipLaunchKernelGGL(k_diff_force_euler, dim3(dgrid((int64_t)n * kDiffSub)), dim3(256), 0, st, p, a, XP, VR, L, nn,
                     d.WP, Xn, Vn);
}
void launch_diff_adjoint(const DevParams &p, const DevPtrs &d, int n, int cap, float dt, float B,
                         float alpha, float hc0, const float4 *X, const float4 *V,
                         const float *rho, const float *prs, const uint32_t *L,
                         const uint32_t *nn, float4 *XB, float4 *VB, float4 *AB, float4 *XR,
                         float4 *VP, float4 *XRB, double *BB, double *AA, hipStream_t st) {
  if (n == 0) return;
  const DiffArgs a = dargs(n, cap, dt, B, alpha, hc0);
  hipLaunchKernelGGL(k_diff_adj_euler, dim3(dgrid(n)), dim3(256), 0, st, a, XB, VB, AB, X, V, rho,
                     prs, XR, VP);
  hipLaunchKernelGGL(k_diff_adj_force, dim3(dgrid((int64_t)n * kDiffSub)), dim3(256), 0, st, p, a, XR, VP, L, nn,
                     d.WP, AB, XB, VB, XRB, BB, AA);
  hipLaunchKernelGGL(k_diff_adj_density, dim3(dgrid((int64_t)n * kDiffSub)), dim3(256), 0, st, p, a, XRB, L, nn,
                     d.WP, XB);
}
void launch_diff_reduce(int n, const double *BB, const double *AA, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_diff_reduce, dim3(1), dim3(256), 0, st, n, BB, AA, out);
}

}  // namespace rts
