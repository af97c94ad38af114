// HIP kernels of one WCSPH regional-time-stepping base step on gfx950.
//
// Order of one base step (Algorithm 1 of Goswami & Batty, with the Serna
// corrector of the step that ends now placed before the predictor of the
// next one, as the predictor-corrector equations of Section 4.1 require):
//   key_hist        block key of every particle + per-block arrival counts
//   scan            exclusive scan of the counts (decoupled look-back)
//   scatter         block-grouped previous indices
//   cell_gather     one wave per block: canonical (stable) order, gather of
//                   the SoA state, block maxima of |v|^2 and |a|^2, block level
//                   from Eq. 2-3 (Section 3.1)
//   rmin_flags      one wave per block: R_min smoothing (Section 4.2), particle
//                   validity / compute / pre-emption, active-list compaction
//   search_density  active particles: neighbours from the 27 surrounding
//                   blocks (list written), density and Tait pressure
//   force           active particles: pressure + viscosity + gravity
//   correct_predict all particles: corrector for the active ones, then the
//                   predictor of the next base step
//
// Every float comparison that decides an integer (block key, neighbour
// predicate, block level) is evaluated with contraction off and a fixed
// operation order, so the structure is reproducible bit for bit on the CPU.
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

// Squared distance with the same fixed order, from xj - xi per axis.
__device__ inline float dist2_exact(float xi, float yi, float zi, float xj, float yj, float zj) {
#pragma clang fp contract(off)
  float dx = xj - xi, dy = yj - yi, dz = zj - zi;
  float xx = dx * dx, yy = dy * dy, zz = dz * dz;
  float s = xx + yy;
  return s + zz;
}

// Cubic spline shape w(q) and its derivative (support q < 2).
__device__ inline float w_shape(float q) {
  if (q < 1.0f) return 1.0f + q * q * (-1.5f + 0.75f * q);
  if (q < 2.0f) {
    float t = 2.0f - q;
    return 0.25f * t * t * t;
  }
  return 0.0f;
}
__device__ inline float dw_shape(float q) {
  if (q < 1.0f) return q * (-3.0f + 2.25f * q);
  if (q < 2.0f) {
    float t = 2.0f - q;
    return -0.75f * t * t;
  }
  return 0.0f;
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

// ---------------------------------------------------------------------------
// key + histogram
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_key_hist(DevParams p, const float4 *__restrict__ P,
                                                 const uint32_t *__restrict__ ids,
                                                 uint32_t *__restrict__ keyold,
                                                 uint32_t *__restrict__ rank,
                                                 uint32_t *__restrict__ count, DevCtrl *ctrl,
                                                 DevScalars *S) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    // per-step control words; every later kernel of the step sees them
    ctrl->epoch += 1u;
    ctrl->scan_ticket = 0u;
    S->n_act = 0u;
    S->amax2_bits = 0u;
    S->err_bits_last = 0u;
    S->inter_last = 0ull;
    for (int l = 0; l < kMaxLevels; ++l) S->hist[l] = 0;
    S->dt_prev = S->dt_next;
  }
  if (i >= p.n) return;
  float4 x = P[i];
  bool bad = !(isfinite(x.x) && isfinite(x.y) && isfinite(x.z));
  // domain check in float against the grid extent
  bad = bad || x.x < p.o[0] || x.y < p.o[1] || x.z < p.o[2] || x.x > p.dmax[0] ||
        x.y > p.dmax[1] || x.z > p.dmax[2];
  if (bad) set_status(S, RTS_E_NUMERICAL, (int32_t)ids[i]);
  uint32_t k = key_of(p, block_of(p, x.x, x.y, x.z));
  keyold[i] = k;
  rank[i] = atomicAdd(&count[k], 1u);
}

// ---------------------------------------------------------------------------
// exclusive scan, single pass with decoupled look-back
// (Merrill & Garland, "Single-pass Parallel Prefix Scan with Decoupled
// Look-back", 2016).  Tiles take tickets in launch order so every tile's
// predecessors have started; status words carry the step's epoch so they
// never need clearing.  Reading a count also clears it for the next sort.
// ---------------------------------------------------------------------------
constexpr unsigned long long kFlagAgg = 1ull, kFlagPre = 2ull;
__device__ inline unsigned long long pack_status(uint32_t epoch, unsigned long long flag,
                                                 uint32_t v) {
  return ((unsigned long long)(epoch & 0x3FFFFFFFu) << 34) | (flag << 32) | v;
}

__global__ void __launch_bounds__(256) k_scan(uint32_t *__restrict__ count,
                                             uint32_t *__restrict__ start, int nb,
                                             unsigned long long *__restrict__ tiles,
                                             DevCtrl *ctrl, DevScalars *S) {
  __shared__ uint32_t s_tile, s_prefix;
  __shared__ uint32_t s_wave[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) s_tile = atomicAdd(&ctrl->scan_ticket, 1u);
  __syncthreads();
  const uint32_t tile = s_tile;
  const uint32_t epoch = ctrl->epoch;
  const int base = (int)tile * kScanTile + tid * 4;
  uint32_t v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int idx = base + k;
    v[k] = idx < nb ? count[idx] : 0u;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (base + k < nb) count[base + k] = 0u;
  uint32_t incl[4];
  incl[0] = v[0];
  incl[1] = incl[0] + v[1];
  incl[2] = incl[1] + v[2];
  incl[3] = incl[2] + v[3];
  uint32_t t = incl[3];
  // inclusive scan of per-thread totals across the wave
  uint32_t x = t;
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = (uint32_t)__shfl_up((int)x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_wave[wave] = x;
  __syncthreads();
  uint32_t wave_off = 0, total = 0;
  for (int w = 0; w < 4; ++w) {
    if (w < wave) wave_off += s_wave[w];
    total += s_wave[w];
  }
  uint32_t thread_excl = wave_off + x - t;
  if (tid == 0) {
    uint32_t excl = 0;
    if (tile == 0) {
      __hip_atomic_store(&tiles[0], pack_status(epoch, kFlagPre, total), __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_AGENT);
    } else {
      __hip_atomic_store(&tiles[tile], pack_status(epoch, kFlagAgg, total), __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_AGENT);
      int j = (int)tile - 1;
      uint32_t spins = 0;
      while (j >= 0) {
        unsigned long long w =
            __hip_atomic_load(&tiles[j], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        unsigned long long flag = (w >> 32) & 3ull;
        uint32_t ep = (uint32_t)(w >> 34);
        if (ep != (epoch & 0x3FFFFFFFu) || flag == 0ull) {
          if (++spins > (1u << 24)) {  // predecessors always finish; this bound is a guard
            set_status(S, RTS_E_DEVICE, -1);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        excl += (uint32_t)(w & 0xFFFFFFFFull);
        if (flag == kFlagPre) break;
        --j;
      }
      __hip_atomic_store(&tiles[tile], pack_status(epoch, kFlagPre, excl + total),
                         __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    s_prefix = excl;
  }
  __syncthreads();
  const uint32_t off = s_prefix + thread_excl;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int idx = base + k;
    if (idx < nb) start[idx] = off + incl[k] - v[k];
    if (idx == nb - 1) start[nb] = off + incl[k];
  }
}

__global__ void k_prep_scan(DevCtrl *ctrl) {
  ctrl->epoch += 1u;
  ctrl->scan_ticket = 0u;
}

// ---------------------------------------------------------------------------
// scatter into blocks (arrival order within a block; canonicalised next)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_scatter(int n, const uint32_t *__restrict__ keyold,
                                                const uint32_t *__restrict__ rank,
                                                const uint32_t *__restrict__ start,
                                                uint32_t *__restrict__ tmp, DevScalars *S) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t d = start[keyold[i]] + rank[i];
  if (d < (uint32_t)n)
    tmp[d] = (uint32_t)i;
  else
    set_status(S, RTS_E_DEVICE, -1);  // inconsistent block starts: never write out of range
}

// Rank of element k among the n distinct values s[0..n): the stable position
// of an index inside its block.
__device__ inline uint32_t rank_in(const uint32_t *s, int n, uint32_t val) {
  uint32_t r = 0;
  for (int m = 0; m < n; ++m) r += (s[m] < val) ? 1u : 0u;
  return r;
}

// ---------------------------------------------------------------------------
// one wave per block: canonical order, gather, block maxima, block level
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_cell_gather(
    DevParams p, const uint32_t *__restrict__ start, const uint32_t *__restrict__ tmp,
    uint32_t *__restrict__ perm, uint32_t *__restrict__ key,
    const float4 *__restrict__ Pi, const float4 *__restrict__ Vi, const float4 *__restrict__ Ai,
    const uint32_t *__restrict__ Mi, const uint32_t *__restrict__ Ii, float4 *__restrict__ Po,
    float4 *__restrict__ Vo, float4 *__restrict__ Ao, uint32_t *__restrict__ Mo,
    uint32_t *__restrict__ Io, uint8_t *__restrict__ lraw, DevScalars *S) {
  __shared__ uint32_t s_idx[kCellMax];
  const int b = blockIdx.x, lane = threadIdx.x;
  const uint32_t s0 = start[b];
  const uint32_t s1 = start[b + 1];
  if (s1 <= s0 || s1 > (uint32_t)p.n) {
    if (lane == 0) {
      lraw[b] = kEmpty;
      if (s1 < s0 || s1 > (uint32_t)p.n) set_status(S, RTS_E_DEVICE, -1);
    }
    return;
  }
  const int n = (int)(s1 - s0);
  const bool canon = n <= kCellMax;
  if (!canon && lane == 0) set_status(S, RTS_E_CAPACITY, -1);
  if (canon)
    for (int k = lane; k < n; k += 64) s_idx[k] = tmp[s0 + k];
  __syncthreads();
  float v2m = 0.0f, a2m = 0.0f;
  for (int k = lane; k < n; k += 64) {
    uint32_t src = canon ? s_idx[k] : tmp[s0 + k];
    uint32_t dst = s0 + (canon ? rank_in(s_idx, n, src) : (uint32_t)k);
    if (src >= (uint32_t)p.n) {
      set_status(S, RTS_E_DEVICE, -1);
      continue;
    }
    perm[dst] = src;
    key[dst] = (uint32_t)b;
    float4 x = Pi[src], v = Vi[src], a = Ai[src];
    Po[dst] = x;
    Vo[dst] = v;
    Ao[dst] = a;
    Mo[dst] = Mi[src];
    Io[dst] = Ii[src];
    v2m = fmaxf(v2m, norm2_exact(v.x, v.y, v.z));
    a2m = fmaxf(a2m, norm2_exact(a.x, a.y, a.z));
  }
  v2m = wave_max(v2m);
  a2m = wave_max(a2m);
  if (lane == 0) {
    // Section 3.1: the block takes the largest step whose Eq. 2 and Eq. 3
    // bounds hold for its fastest and most accelerated particles.
    int l = 0;
    while (l + 1 <= p.lmax && v2m <= p.TV[l + 1] && a2m <= p.TA[l + 1]) ++l;
    lraw[b] = (uint8_t)l;
  }
}

// ---------------------------------------------------------------------------
// one wave per block: R_min, particle flags, active-list compaction
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_rmin_flags(DevParams p, const uint32_t *__restrict__ start,
                                                  const uint8_t *__restrict__ lraw,
                                                  uint8_t *__restrict__ lvl,
                                                  uint32_t *__restrict__ M,
                                                  uint32_t *__restrict__ act, DevScalars *S,
                                                  int do_flags) {
  const int b = blockIdx.x, lane = threadIdx.x;
  const uint32_t own = lraw[b];
  if (own == kEmpty) {
    if (lane == 0) lvl[b] = kEmpty;
    return;
  }
  // R_min (Section 4.2): the smaller step of any occupied neighbour wins.
  uint32_t l = own;
  if (lane < 27) {
    int3 c = coords_of(p, (uint32_t)b);
    int dx = lane % 3 - 1, dy = (lane / 3) % 3 - 1, dz = lane / 9 - 1;
    int x = c.x + dx, y = c.y + dy, z = c.z + dz;
    if (x >= 0 && y >= 0 && z >= 0 && x < p.nc[0] && y < p.nc[1] && z < p.nc[2])
      l = lraw[(uint32_t)(x + p.nc[0] * (y + p.nc[1] * z))];  // 0xFF never wins
  } else {
    l = 0xFFu;
  }
  l = min(wave_min_u32(l), own);
  if (lane == 0) lvl[b] = (uint8_t)l;
  if (!do_flags) return;
  const uint32_t s0 = start[b];
  const int n = (int)(start[b + 1] - s0);
  for (int k0 = 0; k0 < n; k0 += 64) {
    int k = k0 + lane;
    bool comp = false;
    uint32_t i = s0 + (uint32_t)k;
    if (k < n) {
      // Algorithm 1: decrement validity; active when it ran out or the
      // block's step differs (pre-emption); an active particle adopts the
      // block's step and a validity of 2^level base steps.
      uint32_t m = M[i];
      int32_t val = meta_validity(m) - 1;
      uint32_t lev = meta_level(m);
      comp = val <= 0 || lev != l;
      if (comp) {
        lev = l;
        val = 1 << l;
      }
      M[i] = meta_pack(lev, comp ? 1u : 0u, meta_age(m), val);
    }
    unsigned long long mask = __ballot(comp);
    uint32_t cnt = (uint32_t)__popcll(mask);
    uint32_t off = 0;
    if (lane == 0 && cnt) off = atomicAdd(&S->n_act, cnt);
    off = (uint32_t)__shfl((int)off, 0, 64);
    if (comp) {
      unsigned long long below = mask & ((1ull << lane) - 1ull);
      act[off + (uint32_t)__popcll(below)] = i;
    }
  }
  if (lane == 0) atomicAdd(&S->hist[l], n);
}

// ---------------------------------------------------------------------------
// neighbour search + density + Tait pressure (active particles)
// ---------------------------------------------------------------------------
// Tait pressure from the density deviation d = rho/rho0 - 1, with
// (1 + d)^7 - 1 expanded in d (gamma = 7) so that nothing cancels.
__device__ inline float tait_from_dev(const DevParams &p, float d) {
  float poly = 7.0f + d * (21.0f + d * (35.0f + d * (35.0f + d * (21.0f + d * (7.0f + d)))));
  float pr = p.B * d * poly;
  if (p.clamp_p && pr < 0.0f) pr = 0.0f;
  return pr;
}

template <bool kWalls>
__device__ inline void scan_rows(const DevParams &p, int3 c, uint32_t self, float xi, float yi,
                                 float zi, const uint32_t *__restrict__ start,
                                 const float4 *__restrict__ X, uint32_t lim, uint32_t tag,
                                 uint32_t *__restrict__ nbr, uint32_t i, int &cnt, float &sum,
                                 float &comp) {
  const int x0 = max(c.x - 1, 0), x1 = min(c.x + 1, p.nc[0] - 1);
  for (int dz = -1; dz <= 1; ++dz) {
    const int z = c.z + dz;
    if (z < 0 || z >= p.nc[2]) continue;
    for (int dy = -1; dy <= 1; ++dy) {
      const int y = c.y + dy;
      if (y < 0 || y >= p.nc[1]) continue;
      const uint32_t row = (uint32_t)p.nc[0] * ((uint32_t)y + (uint32_t)p.nc[1] * (uint32_t)z);
      const uint32_t j0 = start[row + (uint32_t)x0];
      const uint32_t j1 = min(start[row + (uint32_t)x1 + 1u], lim);
      for (uint32_t j = j0; j < j1; ++j) {
        if (!kWalls && j == self) continue;
        float4 q = X[j];
        float d2 = dist2_exact(xi, yi, zi, q.x, q.y, q.z);
        if (d2 < p.r2f) {
          if (cnt < p.kcap) nbr[(size_t)cnt * (size_t)p.ncap + i] = j | tag;
          ++cnt;
          float w = w_shape(sqrtf(d2) * p.inv_h);
          // Kahan-compensated sum of W (in units of sigma)
          float y2 = w - comp;
          float t = sum + y2;
          comp = (t - sum) - y2;
          sum = t;
        }
      }
    }
  }
}

__global__ void __launch_bounds__(256) k_search_density(
    DevParams p, const uint32_t *__restrict__ act, const uint32_t *__restrict__ key,
    const uint32_t *__restrict__ start, float4 *__restrict__ P, float4 *__restrict__ V,
    float *__restrict__ pres, uint32_t *__restrict__ nnb, uint32_t *__restrict__ nbr,
    const uint32_t *__restrict__ wstart, const float4 *__restrict__ WP,
    const uint32_t *__restrict__ ids, DevScalars *S) {
  const uint32_t nact = S->n_act;
  const int lane = threadIdx.x & 63;
  uint32_t inter = 0, cmax = 0;
  for (uint32_t slot = blockIdx.x * blockDim.x + threadIdx.x;
       slot - lane < nact;  // whole waves iterate together
       slot += gridDim.x * blockDim.x) {
    const bool live = slot < nact;
    if (live) {
      const uint32_t i = act[slot];
      const float4 xi = P[i];
      const int3 c = coords_of(p, key[i]);
      int cnt = 0;
      float sum = 0.0f, comp = 0.0f;
      scan_rows<false>(p, c, i, xi.x, xi.y, xi.z, start, P, (uint32_t)p.n, 0u, nbr, i, cnt, sum,
                       comp);
      if (p.nw > 0)
        scan_rows<true>(p, c, 0xFFFFFFFFu, xi.x, xi.y, xi.z, wstart, WP, (uint32_t)p.nw, kWallBit,
                        nbr, i, cnt, sum, comp);
      if (cnt > p.kcap) set_status(S, RTS_E_CAPACITY, (int32_t)ids[i]);
      // rho/rho0 - 1 = (m sigma / rho0) (sum - C) with C = rho0/(m sigma) - 1,
      // sum = neighbour sum of the kernel shape (self excluded), carried as
      // sum - comp; the difference is formed before any rounding to rho.
      const float dev = p.kms * ((sum - p.c_hi) - (comp + p.c_lo));
      const float rho = p.rho0 + p.rho0 * dev;
      const float pr = tait_from_dev(p, dev);
      reinterpret_cast<float *>(&P[i])[3] = rho;
      reinterpret_cast<float *>(&V[i])[3] = pr / (rho * rho);
      pres[i] = pr;
      nnb[i] = (uint32_t)min(cnt, p.kcap);
      inter += (uint32_t)cnt;
      cmax = max(cmax, (uint32_t)cnt);
    }
  }
  inter = wave_sum_u32(inter);
  cmax = wave_max_u32(cmax);
  if (lane == 0) {
    if (inter) atomicAdd(&S->inter_last, (unsigned long long)inter);
    atomicMax(&S->nbr_max, cmax);
  }
}

// ---------------------------------------------------------------------------
// forces (active particles)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_force(DevParams p, const uint32_t *__restrict__ act,
                                              const float4 *__restrict__ P,
                                              const float4 *__restrict__ V,
                                              const uint32_t *__restrict__ nnb,
                                              const uint32_t *__restrict__ nbr,
                                              const float4 *__restrict__ WP,
                                              float4 *__restrict__ anew, DevScalars *S) {
  const uint32_t nact = S->n_act;
  const int lane = threadIdx.x & 63;
  float a2max = 0.0f;
  const float coefg = p.sigma * p.inv_h;  // dW/dr = sigma / h * w'(q)
  for (uint32_t slot = blockIdx.x * blockDim.x + threadIdx.x; slot - lane < nact;
       slot += gridDim.x * blockDim.x) {
    if (slot < nact) {
      const uint32_t i = act[slot];
      const float4 pi = P[i], vi = V[i];
      const float rhoi = pi.w, pri = vi.w;
      float ax = 0.0f, ay = 0.0f, az = 0.0f;
      const int cnt = (int)nnb[i];
      for (int k = 0; k < cnt; ++k) {
        const uint32_t j = nbr[(size_t)k * (size_t)p.ncap + i];
        float xj, yj, zj, vxj, vyj, vzj, rhoj, prj;
        if (j & kWallBit) {
          // static wall particle: at rest, density mirrored, pressure mirrored
          // plus the hydrostatic difference, clamped at zero
          const float4 q = WP[j & ~kWallBit];
          xj = q.x; yj = q.y; zj = q.z;
          vxj = vyj = vzj = 0.0f;
          rhoj = rhoi;
          const float gd = p.g[0] * (xj - pi.x) + p.g[1] * (yj - pi.y) + p.g[2] * (zj - pi.z);
          prj = fmaxf(pri + gd / rhoi, 0.0f);
        } else {
          const float4 q = P[j], u = V[j];
          xj = q.x; yj = q.y; zj = q.z; rhoj = q.w;
          vxj = u.x; vyj = u.y; vzj = u.z; prj = u.w;
        }
        const float dx = pi.x - xj, dy = pi.y - yj, dz = pi.z - zj;
        const float r2 = dx * dx + dy * dy + dz * dz;
        if (r2 <= 0.0f) continue;
        const float rinv = rsqrtf(r2);
        const float r = r2 * rinv;
        const float f = coefg * dw_shape(r * p.inv_h) * rinv;  // gradW = f * x_ij
        float coef = pri + prj;
        const float vx = (vi.x - vxj) * dx + (vi.y - vyj) * dy + (vi.z - vzj) * dz;
        if (vx < 0.0f) {
          const float nu = p.visc_num / (rhoi + rhoj);
          coef -= nu * vx / (r2 + p.visc_eps_h2);
        }
        const float s = -p.mass * coef * f;
        ax += s * dx;
        ay += s * dy;
        az += s * dz;
      }
      ax += p.g[0];
      ay += p.g[1];
      az += p.g[2];
      anew[i] = make_float4(ax, ay, az, 0.0f);
      a2max = fmaxf(a2max, ax * ax + ay * ay + az * az);
    }
  }
  a2max = wave_max(a2max);
  if (lane == 0 && a2max > 0.0f) atomicMax(&S->amax2_bits, __float_as_uint(a2max));
}

// ---------------------------------------------------------------------------
// corrector (active) + predictor (all)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_correct_predict(DevParams p, float4 *__restrict__ P,
                                                        float4 *__restrict__ V,
                                                        float4 *__restrict__ A,
                                                        uint32_t *__restrict__ M,
                                                        const float4 *__restrict__ anew,
                                                        DevScalars *S) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  // step length: fixed, or the adaptive comparator's
  double dtd = p.dt_base;
  if (p.mode == RTS_MODE_GLOBAL_ADAPTIVE) {
    dtd = p.dt_cfl;
    const float a2 = __uint_as_float(S->amax2_bits);
    if (a2 > 0.0f) {
      const double df = sqrt(p.lf2r / sqrt((double)a2));
      if (df < dtd) dtd = df;
    }
  }
  const float dt = (float)dtd;
  float err = 0.0f;
  if (i < p.n) {
    float4 x = P[i], v = V[i], a = A[i];
    uint32_t m = M[i];
    uint32_t age = meta_age(m);
    if (meta_compute(m)) {
      const float4 an = anew[i];
      if (p.serna_correct) {
        const float dtau = p.mode == RTS_MODE_GLOBAL_ADAPTIVE ? (float)S->dt_prev
                                                              : (float)age * p.dt_base;
        const float cx = dtau * dtau * (1.0f / 6.0f), cv = dtau * 0.5f;
        const float dax = an.x - a.x, day = an.y - a.y, daz = an.z - a.z;
        x.x += dax * cx; x.y += day * cx; x.z += daz * cx;
        v.x += dax * cv; v.y += day * cv; v.z += daz * cv;
      }
      a.x = an.x; a.y = an.y; a.z = an.z;
      age = 0;
    }
    const float h2 = 0.5f * dt * dt;
    x.x += v.x * dt + a.x * h2;
    x.y += v.y * dt + a.y * h2;
    x.z += v.z * dt + a.z * h2;
    v.x += a.x * dt;
    v.y += a.y * dt;
    v.z += a.z * dt;
    age = min(age + 1u, 0x7FFu);
    P[i] = x;
    V[i] = v;
    A[i] = a;
    M[i] = meta_pack(meta_level(m), meta_compute(m), age, meta_validity(m));
    err = fmaxf((x.w - p.rho0) / p.rho0, 0.0f);
  }
  err = wave_max(err);
  if (lane == 0 && err > 0.0f) {
    atomicMax(&S->err_bits_last, __float_as_uint(err));
    atomicMax(&S->err_bits_run, __float_as_uint(err));
  }
  if (i == 0) {
    S->dt_next = dtd;
    S->time += dtd;
    S->step += 1;
    S->active_total += S->n_act;
    S->inter_total += S->inter_last;
  }
}

// ---------------------------------------------------------------------------
// state in / out, walls
// ---------------------------------------------------------------------------
__global__ void k_set_state(DevParams p, const float *__restrict__ pos,
                            const float *__restrict__ vel, float4 *P, float4 *V, float4 *A,
                            uint32_t *M, uint32_t *ID, float *pres) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  size_t n = (size_t)p.n;
  P[i] = make_float4(pos[i], pos[n + i], pos[2 * n + i], p.rho0);
  V[i] = vel ? make_float4(vel[i], vel[n + i], vel[2 * n + i], 0.0f)
             : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  A[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  M[i] = meta_pack(0xFu, 0u, 0u, 0);
  ID[i] = (uint32_t)i;
  pres[i] = 0.0f;
}

__global__ void k_get_state(DevParams p, const float4 *P, const float4 *V, const float4 *A,
                            const uint32_t *M, const uint32_t *ID, const float *pres, float *pos,
                            float *vel, float *acc, float *rho, float *po, uint8_t *level) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  size_t n = (size_t)p.n;
  uint32_t c = ID[i];
  float4 x = P[i];
  if (pos) { pos[c] = x.x; pos[n + c] = x.y; pos[2 * n + c] = x.z; }
  if (vel) { float4 v = V[i]; vel[c] = v.x; vel[n + c] = v.y; vel[2 * n + c] = v.z; }
  if (acc) { float4 a = A[i]; acc[c] = a.x; acc[n + c] = a.y; acc[2 * n + c] = a.z; }
  if (rho) rho[c] = x.w;
  if (po) po[c] = V[i].w * x.w * x.w;  // V.w holds p / rho^2
  if (level) level[c] = (uint8_t)meta_level(M[i]);
}

__global__ void k_wall_keys(DevParams p, const float *__restrict__ pos, uint32_t *wkey,
                            uint32_t *wrank, uint32_t *count) {
  int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= p.nw) return;
  size_t n = (size_t)p.nw;
  uint32_t k = key_of(p, block_of(p, pos[w], pos[n + w], pos[2 * n + w]));
  wkey[w] = k;
  wrank[w] = atomicAdd(&count[k], 1u);
}

__global__ void __launch_bounds__(64) k_wall_gather(DevParams p, const uint32_t *__restrict__ start,
                                                   const uint32_t *__restrict__ tmp,
                                                   const float *__restrict__ pos, float4 *WP,
                                                   uint32_t *WID, DevScalars *S) {
  __shared__ uint32_t s_idx[kCellMax];
  const int b = blockIdx.x, lane = threadIdx.x;
  const uint32_t s0 = start[b];
  const uint32_t s1 = start[b + 1];
  if (s1 <= s0 || s1 > (uint32_t)p.nw) {
    if (lane == 0 && (s1 < s0 || s1 > (uint32_t)p.nw)) set_status(S, RTS_E_DEVICE, -1);
    return;
  }
  const int n = (int)(s1 - s0);
  const bool canon = n <= kCellMax;
  if (!canon && lane == 0) set_status(S, RTS_E_CAPACITY, -1);
  if (canon)
    for (int k = lane; k < n; k += 64) s_idx[k] = tmp[s0 + k];
  __syncthreads();
  size_t nw = (size_t)p.nw;
  for (int k = lane; k < n; k += 64) {
    uint32_t src = canon ? s_idx[k] : tmp[s0 + k];
    uint32_t dst = s0 + (canon ? rank_in(s_idx, n, src) : (uint32_t)k);
    if (src >= (uint32_t)p.nw) {
      set_status(S, RTS_E_DEVICE, -1);
      continue;
    }
    WP[dst] = make_float4(pos[src], pos[nw + src], pos[2 * nw + src], 0.0f);
    WID[dst] = src;
  }
}

__global__ void k_reset_scalars(DevScalars *S) {
  DevScalars z = {};
  z.bad_index = -1;
  *S = z;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(int n, int t) { return (unsigned)((n + t - 1) / t); }

void launch_key_hist(const DevParams &p, const DevPtrs &d, int cur, hipStream_t st) {
  hipLaunchKernelGGL(k_key_hist, dim3(blocks_for(p.n > 0 ? p.n : 1, 256)), dim3(256), 0, st, p,
                     d.P[cur], d.ID[cur], d.KEYOLD, d.RANK, d.COUNT, d.CTRL, d.S);
}
void launch_prep_scan(DevCtrl *ctrl, hipStream_t st) {
  hipLaunchKernelGGL(k_prep_scan, dim3(1), dim3(1), 0, st, ctrl);
}
void launch_scan(const DevParams &p, uint32_t *count, uint32_t *start, int nb,
                 unsigned long long *tiles, DevCtrl *ctrl, DevScalars *S, hipStream_t st) {
  (void)p;
  hipLaunchKernelGGL(k_scan, dim3(blocks_for(nb, kScanTile)), dim3(256), 0, st, count, start, nb,
                     tiles, ctrl, S);
}
void launch_scatter(const DevParams &p, const DevPtrs &d, hipStream_t st) {
  if (p.n == 0) return;
  hipLaunchKernelGGL(k_scatter, dim3(blocks_for(p.n, 256)), dim3(256), 0, st, p.n, d.KEYOLD,
                     d.RANK, d.CELL_START, d.TMP, d.S);
}
void launch_cell_gather(const DevParams &p, const DevPtrs &d, int cur, hipStream_t st) {
  int nx = cur ^ 1;
  hipLaunchKernelGGL(k_cell_gather, dim3((unsigned)p.nb), dim3(64), 0, st, p, d.CELL_START, d.TMP,
                     d.PERM, d.KEY, d.P[cur], d.V[cur], d.A[cur], d.M[cur], d.ID[cur], d.P[nx],
                     d.V[nx], d.A[nx], d.M[nx], d.ID[nx], d.LRAW, d.S);
}
void launch_rmin_flags(const DevParams &p, const DevPtrs &d, int cur, int do_flags,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_rmin_flags, dim3((unsigned)p.nb), dim3(64), 0, st, p, d.CELL_START,
                     d.LRAW, d.LVL, d.M[cur], d.ACT, d.S, do_flags);
}
void launch_search_density(const DevParams &p, const DevPtrs &d, int cur, int grid,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_search_density, dim3((unsigned)grid), dim3(256), 0, st, p, d.ACT, d.KEY,
                     d.CELL_START, d.P[cur], d.V[cur], d.PRES, d.NNB, d.NBR, d.WCELL_START, d.WP,
                     d.ID[cur], d.S);
}
void launch_force(const DevParams &p, const DevPtrs &d, int cur, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_force, dim3((unsigned)grid), dim3(256), 0, st, p, d.ACT, d.P[cur],
                     d.V[cur], d.NNB, d.NBR, d.WP, d.ANEW, d.S);
}
void launch_correct_predict(const DevParams &p, const DevPtrs &d, int cur, hipStream_t st) {
  hipLaunchKernelGGL(k_correct_predict, dim3(blocks_for(p.n > 0 ? p.n : 1, 256)), dim3(256), 0,
                     st, p, d.P[cur], d.V[cur], d.A[cur], d.M[cur], d.ANEW, d.S);
}
void launch_set_state(const DevParams &p, const DevPtrs &d, int cur, const float *pos,
                      const float *vel, hipStream_t st) {
  if (p.n == 0) return;
  hipLaunchKernelGGL(k_set_state, dim3(blocks_for(p.n, 256)), dim3(256), 0, st, p, pos, vel,
                     d.P[cur], d.V[cur], d.A[cur], d.M[cur], d.ID[cur], d.PRES);
}
void launch_get_state(const DevParams &p, const DevPtrs &d, int cur, float *pos, float *vel,
                      float *acc, float *rho, float *pres, uint8_t *level, hipStream_t st) {
  if (p.n == 0) return;
  hipLaunchKernelGGL(k_get_state, dim3(blocks_for(p.n, 256)), dim3(256), 0, st, p, d.P[cur],
                     d.V[cur], d.A[cur], d.M[cur], d.ID[cur], d.PRES, pos, vel, acc, rho, pres,
                     level);
}
void launch_wall_sort(const DevParams &p, const DevPtrs &d, const float *pos, hipStream_t st) {
  launch_prep_scan(d.CTRL, st);
  if (p.nw > 0)
    hipLaunchKernelGGL(k_wall_keys, dim3(blocks_for(p.nw, 256)), dim3(256), 0, st, p, pos, d.WKEY,
                       d.WRANK, d.COUNT);
  launch_scan(p, d.COUNT, d.WCELL_START, p.nb, d.TILES, d.CTRL, d.S, st);
  if (p.nw > 0) {
    hipLaunchKernelGGL(k_scatter, dim3(blocks_for(p.nw, 256)), dim3(256), 0, st, p.nw, d.WKEY,
                       d.WRANK, d.WCELL_START, d.WTMP, d.S);
    hipLaunchKernelGGL(k_wall_gather, dim3((unsigned)p.nb), dim3(64), 0, st, p, d.WCELL_START,
                       d.WTMP, pos, d.WP, d.WID, d.S);
  }
}
void launch_reset_scalars(DevScalars *S, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_scalars, dim3(1), dim3(1), 0, st, S);
}

}  // namespace rts
