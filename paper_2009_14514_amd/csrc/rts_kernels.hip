// HIP kernels of one WCSPH regional-time-stepping base step on gfx950.
//
// Order of one base step (Algorithm 1 of Goswami & Batty, with the Serna
// corrector of the step that ends now placed before the predictor of the
// next one, as the predictor-corrector equations of Section 4.1 require):
//   key_hist        block key of every particle + per-block arrival counts
//   scan            exclusive scans (decoupled look-back) of the counts and of
//                   the occupied-block flags: block starts, occupied-block list
//   scatter         block-grouped previous indices
//   cell_gather     one wave per occupied block: canonical (stable) order, SoA
//                   gather, block maxima of |v|^2 and |a|^2, block level from
//                   Eq. 2-3 (Section 3.1)
//   rmin_flags      one wave per occupied block: R_min smoothing (Section 4.2),
//                   particle validity / compute / pre-emption (Algorithm 1)
//   search_density  one workgroup per active block: the 27 surrounding
//                   blocks are staged in LDS once; a wave tests a few
//                   particles at a time against chunks of 64 candidates (a
//                   candidate per lane) and writes each particle's neighbour
//                   list in canonical order from the lane masks; then sums
//                   the density over the lists; Tait pressure
//   force           one workgroup per active block: candidates' position,
//                   velocity, density and pressure staged in LDS; pressure +
//                   viscosity + gravity over the lists, a particle's entries
//                   shared evenly by its lanes
//   step_stats      per-step counters and the step length
//   correct_predict all particles: corrector for the active ones, then the
//                   predictor of the next base step
// With a fixed base step (RTS, global fixed) the last two are one launch,
// stats_correct_predict, which also does the next step's key_hist on the
// predicted positions; key_hist itself then runs only before the first step
// after the particles change, and for the adaptive comparator.
//
// Every float comparison that decides an integer (block key, neighbour
// predicate, block level) is evaluated with contraction off and a fixed
// operation order, so the structure is reproducible bit for bit on the CPU.
// No floating-point atomics are used; same-address integer atomics are
// limited to one per group of equal keys in a wave.
#include <type_traits>
#include <utility>

#include "rts_device.h"

namespace rts {

// search: 256 or 512 threads (a launch-shape choice)
constexpr int kForceThreads = 512;            // force: 512 / lanes-per-particle particles a pass

// ---------------------------------------------------------------------------
// key + histogram
// ---------------------------------------------------------------------------
// Key of particle i at position x, the domain check, and its slot in the
// histogram of the next sort.  Every lane of the wave must call it (live or
// not).
__device__ inline void bin_particle(const DevParams &p, int i, bool live, float4 x,
                                    const uint32_t *__restrict__ ids,
                                    uint32_t *__restrict__ keyold, uint32_t *__restrict__ rank,
                                    uint32_t *__restrict__ count, DevScalars *S) {
  const int lane = threadIdx.x & 63;
  uint32_t k = 0;
  if (live) {
    bool bad = !(isfinite(x.x) && isfinite(x.y) && isfinite(x.z));
    bad = bad || x.x < p.o[0] || x.y < p.o[1] || x.z < p.o[2] || x.x > p.dmax[0] ||
          x.y > p.dmax[1] || x.z > p.dmax[2];
    if (bad) set_status(S, RTS_E_NUMERICAL, (int32_t)ids[i]);
    k = key_of(p, block_of(p, x.x, x.y, x.z));
    keyold[i] = k;
  }
  // Particles arrive in the previous sorted order, so a wave holds few
  // distinct keys: one atomic per distinct key, by the key's first lane, all
  // issued at once; ranks handed out in-wave.
  bool done = !live;
  int leader_of = 0;          // first lane holding this lane's key
  uint32_t below = 0, group = 0;
  unsigned long long todo = __ballot(!done);
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const uint32_t lk = (uint32_t)__shfl((int)k, leader, 64);
    const bool mine = !done && k == lk;
    const unsigned long long same = __ballot(mine);
    if (mine) {
      leader_of = leader;
      below = (uint32_t)__popcll(same & ((1ull << lane) - 1ull));
      done = true;
    }
    if (lane == leader) group = (uint32_t)__popcll(same);
    todo = __ballot(!done);
  }
  uint32_t base = 0;
  if (live && lane == leader_of) base = atomicAdd(&count[k], group);
  base = (uint32_t)__shfl((int)base, leader_of, 64);
  if (live) rank[i] = base + below;
}

// The words a step's kernels count with start from zero (the statistics'
// ticket apart: the fold that consumes it clears it); a fresh epoch for the
// step's scan.
__device__ inline void step_controls_reset(int i, DevCtrl *ctrl, uint32_t *__restrict__ actn) {
  if (i < kActBuckets) actn[i * kActnStride] = 0u;
  if (i == 0) {
    ctrl->epoch += 1u;
    ctrl->scan_ticket = 0u;
    ctrl->search_ticket = 0u;
    ctrl->force_ticket = 0u;
  }
}

__global__ void __launch_bounds__(256) k_key_hist(DevParams p, const float4 *__restrict__ P,
                                                 const uint32_t *__restrict__ ids,
                                                 uint32_t *__restrict__ keyold,
                                                 uint32_t *__restrict__ rank,
                                                 uint32_t *__restrict__ count, DevCtrl *ctrl,
                                                 uint32_t *__restrict__ actn, DevScalars *S) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  step_controls_reset(i, ctrl, actn);
  if (i == 0) {
    ctrl->stats_ticket = 0u;
    S->dt_prev = S->dt_next;
  }
  const bool live = i < p.n;
  bin_particle(p, i, live, live ? P[i] : make_float4(0.0f, 0.0f, 0.0f, 0.0f), ids, keyold, rank,
               count, S);
}

// ---------------------------------------------------------------------------
// exclusive scans, single pass with decoupled look-back
// (Merrill & Garland, "Single-pass Parallel Prefix Scan with Decoupled
// Look-back", 2016).  Tiles take tickets in launch order so every tile's
// predecessors have started; status words carry the scan's epoch so they
// never need clearing.  Reading a count also clears it for the next sort.
// For the fluid grid the same pass scans the occupied-block flags into the
// occupied-block list and marks the levels of empty blocks.
// ---------------------------------------------------------------------------
constexpr unsigned long long kFlagAgg = 1ull, kFlagPre = 2ull;
__device__ inline unsigned long long pack_status(uint32_t epoch, unsigned long long flag,
                                                 uint32_t v) {
  return ((unsigned long long)(epoch & 0x3FFFFFFFu) << 34) | (flag << 32) | v;
}

// One wave of a tile: publish the aggregate, look back, publish the prefix.
// The wave reads the status words of up to 64 predecessors at once (lane l
// the l-th nearest), takes the run of published words up to the nearest
// prefix, and moves on past the run when no prefix is in it.  A status word
// carries everything a successor needs (epoch, flag, value), so the words are
// relaxed device-scope atomics: no cache write-back is needed to publish
// them.  Returns the exclusive prefix in every lane.
__device__ uint32_t look_back(unsigned long long *tiles, uint32_t tile, uint32_t epoch,
                              uint32_t total, DevScalars *S) {
  const int lane = threadIdx.x & 63;
  const uint32_t ep30 = epoch & 0x3FFFFFFFu;
  if (tile == 0) {
    if (lane == 0)
      __hip_atomic_store(&tiles[0], pack_status(epoch, kFlagPre, total), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    return 0;
  }
  if (lane == 0)
    __hip_atomic_store(&tiles[tile], pack_status(epoch, kFlagAgg, total), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  uint32_t excl = 0;
  int hi = (int)tile - 1;  // nearest predecessor not yet added
  uint32_t spins = 0;
  while (true) {
    const int j = hi - lane;
    // below tile 0 reads as a prefix of zero, so every window ends in one
    unsigned long long w = pack_status(epoch, kFlagPre, 0u);
    if (j >= 0) w = __hip_atomic_load(&tiles[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long flag = (w >> 32) & 3ull;
    const bool valid = (uint32_t)(w >> 34) == ep30 && flag != 0ull;
    const unsigned long long inval = __ballot(!valid);
    const unsigned long long pre = __ballot(valid && flag == kFlagPre);
    const int first_inval = inval ? __ffsll((long long)inval) - 1 : 64;
    const int first_pre = pre ? __ffsll((long long)pre) - 1 : 64;
    const int take = first_pre < first_inval ? first_pre + 1 : first_inval;
    if (take > 0) {
      uint32_t v = lane < take ? (uint32_t)(w & 0xFFFFFFFFull) : 0u;
      for (int o = 32; o > 0; o >>= 1) v += (uint32_t)__shfl_xor((int)v, o, 64);
      excl += v;
      if (first_pre < first_inval) break;
      hi -= take;
      continue;
    }
    if (++spins > (1u << 24)) {  // predecessors always finish; this bound is a guard
      if (lane == 0) set_status(S, RTS_E_DEVICE, -1);
      break;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  if (lane == 0)
    __hip_atomic_store(&tiles[tile], pack_status(epoch, kFlagPre, excl + total),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return excl;
}

// Block-wide inclusive scan of one value per thread (256 threads).
__device__ inline uint32_t block_scan_256(uint32_t t, uint32_t *s_wave, uint32_t &total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = t;
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = (uint32_t)__shfl_up((int)x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_wave[wave] = x;
  __syncthreads();
  uint32_t off = 0;
  total = 0;
  for (int w = 0; w < 4; ++w) {
    if (w < wave) off += s_wave[w];
    total += s_wave[w];
  }
  return off + x;
}

__global__ void __launch_bounds__(256) k_scan(uint32_t *__restrict__ count,
                                             uint32_t *__restrict__ start, int nb,
                                             unsigned long long *__restrict__ tiles,
                                             unsigned long long *__restrict__ tiles2,
                                             uint32_t *__restrict__ occ,
                                             uint4 *__restrict__ occr,
                                             uint8_t *__restrict__ lraw,
                                             uint8_t *__restrict__ lvl, DevCtrl *ctrl,
                                             DevScalars *S) {
  __shared__ uint32_t s_tile, s_prefix, s_prefix2;
  __shared__ uint32_t s_wave[4], s_wave2[4];
  const int tid = threadIdx.x;
  if (tid == 0) s_tile = atomicAdd(&ctrl->scan_ticket, 1u);
  __syncthreads();
  const uint32_t tile = s_tile;
  const uint32_t epoch = ctrl->epoch;
  const int base = (int)tile * kScanTile + tid * 4;
  uint32_t v[4], o[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int idx = base + k;
    v[k] = idx < nb ? count[idx] : 0u;
    o[k] = v[k] ? 1u : 0u;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (base + k < nb) count[base + k] = 0u;
  const uint32_t t = v[0] + v[1] + v[2] + v[3];
  const uint32_t t2 = o[0] + o[1] + o[2] + o[3];
  uint32_t total = 0, total2 = 0;
  const uint32_t incl = block_scan_256(t, s_wave, total);
  const uint32_t incl2 = occ ? block_scan_256(t2, s_wave2, total2) : 0u;
  // the two look-backs run in parallel, one wave each
  const int wave = tid >> 6;
  if (wave == 0) {
    const uint32_t pfx = look_back(tiles, tile, epoch, total, S);
    if (tid == 0) s_prefix = pfx;
  } else if (wave == 1 && occ) {
    const uint32_t pfx = look_back(tiles2, tile, epoch, total2, S);
    if (tid == 64) s_prefix2 = pfx;
  }
  __syncthreads();
  uint32_t off = s_prefix + incl - t;
  uint32_t off2 = occ ? s_prefix2 + incl2 - t2 : 0u;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int idx = base + k;
    if (idx < nb) {
      start[idx] = off;
      if (occ) {
        if (v[k]) {
          occ[off2] = (uint32_t)idx;
          occr[off2] = make_uint4((uint32_t)idx, off, off + v[k], 0u);
        } else {
          lraw[idx] = kEmpty;
          lvl[idx] = kEmpty;
        }
      }
    }
    off += v[k];
    off2 += o[k];
    if (idx == nb - 1) {
      start[nb] = off;
      if (occ) S->n_occ = off2;
    }
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
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t d = start[keyold[i]] + rank[i];
  if (d < (uint32_t)n)
    tmp[d] = (uint32_t)i;
  else
    set_status(S, RTS_E_DEVICE, -1);  // inconsistent block starts: never write out of range
}

// Rank of val among the n distinct values s[0..n): the stable position of an
// index inside its block.
__device__ inline uint32_t rank_in(const uint32_t *s, int n, uint32_t val) {
  uint32_t r = 0;
  for (int m = 0; m < n; ++m) r += (s[m] < val) ? 1u : 0u;
  return r;
}

// The same over a shared-memory row padded with 0xFFFFFFFF up to a multiple
// of 16 entries (no value ranks above the padding): four 16-byte reads in
// flight per step instead of one dependent read per entry.
__device__ inline uint32_t rank_in16(const uint4 *s4, int n, uint32_t val) {
  uint32_t r = 0;
  for (int m = 0; m < n; m += 16) {
    uint4 q[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) q[j] = s4[m / 4 + j];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      r += (q[j].x < val ? 1u : 0u) + (q[j].y < val ? 1u : 0u) + (q[j].z < val ? 1u : 0u) +
           (q[j].w < val ? 1u : 0u);
  }
  return r;
}

// ---------------------------------------------------------------------------
// one wave per occupied block: canonical order, gather, block maxima, level
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_cell_gather(
    DevParams p, const uint4 *__restrict__ occr, const uint32_t *__restrict__ tmp,
    uint32_t *__restrict__ perm, uint32_t *__restrict__ key,
    const float4 *__restrict__ Pi, const float4 *__restrict__ Vi, const float4 *__restrict__ Ai,
    const uint32_t *__restrict__ Mi, const uint32_t *__restrict__ Ii, float4 *__restrict__ Po,
    float4 *__restrict__ Vo, float4 *__restrict__ Ao, uint32_t *__restrict__ Mo,
    uint32_t *__restrict__ Io, uint8_t *__restrict__ lraw, DevScalars *S) {
  static_assert(kCellMax % 16 == 0, "rows pad to whole 16-entry groups");
  __shared__ uint4 s_idx_all[4][kCellMax / 4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t *s_idx = reinterpret_cast<uint32_t *>(s_idx_all[wave]);
  const uint32_t nocc = S->n_occ;
  for (uint32_t q = blockIdx.x * 4 + wave; q < nocc; q += gridDim.x * 4) {
    // the block and its range, as the scan left them (one wave-uniform load)
    const uint4 br = occr[__builtin_amdgcn_readfirstlane(q)];
    const uint32_t b = br.x, s0 = br.y, s1 = br.z;
    if (s1 <= s0 || s1 > (uint32_t)p.n) {
      if (lane == 0) {
        lraw[b] = kEmpty;
        set_status(S, RTS_E_DEVICE, -1);
      }
      continue;
    }
    const int n = (int)(s1 - s0);
    const bool canon = n <= kCellMax;
    if (!canon && lane == 0) set_status(S, RTS_E_CAPACITY, -1);
    const int npad = (n + 15) & ~15;
    if (canon)
      for (int k = lane; k < npad; k += 64) s_idx[k] = k < n ? tmp[s0 + k] : 0xFFFFFFFFu;
    // the wave's LDS writes must be visible to the whole wave
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float v2m = 0.0f, a2m = 0.0f;
    const auto move = [&](uint32_t src, uint32_t dst) {
      if (src >= (uint32_t)p.n) {
        set_status(S, RTS_E_DEVICE, -1);
        return;
      }
      perm[dst] = src;
      key[dst] = b;
      const float4 x = Pi[src], v = Vi[src], a = Ai[src];
      Po[dst] = x;
      Vo[dst] = v;
      Ao[dst] = a;
      Mo[dst] = Mi[src];
      Io[dst] = Ii[src];
      v2m = fmaxf(v2m, norm2_exact(v.x, v.y, v.z));
      a2m = fmaxf(a2m, norm2_exact(a.x, a.y, a.z));
    };
    if (canon) {
      for (int k = lane; k < n; k += 64) {
        const uint32_t src = s_idx[k];
        move(src, s0 + rank_in16(s_idx_all[wave], npad, src));
      }
    } else {
      for (int k = lane; k < n; k += 64) move(tmp[s0 + k], s0 + (uint32_t)k);
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
    // s_idx is reused for the next block: all lanes must be done reading it
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// ---------------------------------------------------------------------------
// one wave per occupied block: R_min, particle flags, block active count
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_rmin_flags(DevParams p, const uint4 *__restrict__ occr,
                                                   const uint8_t *__restrict__ lraw,
                                                   uint8_t *__restrict__ lvl,
                                                   uint32_t *__restrict__ M,
                                                   const float4 *__restrict__ P,
                                                   uint4 *__restrict__ blku,
                                                   float *__restrict__ blkerr,
                                                   float *__restrict__ blkamax,
                                                   uint32_t *__restrict__ act,
                                                   uint32_t *__restrict__ actn, DevScalars *S,
                                                   int do_flags) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t nocc = S->n_occ;
  // base steps taken before this one: with phase alignment a particle that
  // takes level l is due again at the next multiple of 2^l
  const uint32_t phase = p.phase_align ? (uint32_t)S->step : 0u;
  for (uint32_t q = blockIdx.x * 4 + wave; q < nocc; q += gridDim.x * 4) {
    // the block and its range, as the scan left them (one wave-uniform load)
    const uint4 br = occr[__builtin_amdgcn_readfirstlane(q)];
    const uint32_t b = br.x;
    const uint32_t own = lraw[b];
    // R_min (Section 4.2): the smaller step of any occupied neighbour wins.
    uint32_t l = 0xFFu;
    if (lane < 27) {
      const int3 c = coords_of(p, b);
      const int x = c.x + lane % 3 - 1, y = c.y + (lane / 3) % 3 - 1, z = c.z + lane / 9 - 1;
      if (x >= 0 && y >= 0 && z >= 0 && x < p.nc[0] && y < p.nc[1] && z < p.nc[2])
        l = lraw[(uint32_t)(x + p.nc[0] * (y + p.nc[1] * z))];  // 0xFF never wins
    }
    l = min(wave_min_u32(l), own);
    if (lane == 0) lvl[b] = (uint8_t)l;
    if (!do_flags) continue;
    const uint32_t s0 = br.y;
    const int n = (int)(br.z - s0);
    uint32_t nact = 0;
    float err = 0.0f;
    for (int k0 = 0; k0 < n; k0 += 64) {
      const int k = k0 + lane;
      bool comp = false;
      if (k < n) {
        // Algorithm 1: decrement validity; active when it ran out or the
        // block's step differs (pre-emption); an active particle adopts the
        // block's step and a validity of 2^level base steps (phase-aligned:
        // up to the next multiple of 2^level).
        const uint32_t i = s0 + (uint32_t)k;
        const uint32_t m = M[i];
        int32_t val = meta_validity(m) - 1;
        uint32_t lev = meta_level(m);
        comp = val <= 0 || lev != l;
        if (comp) {
          lev = l;
          val = (int32_t)((1u << l) - (phase & ((1u << l) - 1u)));
        } else {
          // an inactive particle keeps its last density for this step
          err = fmaxf(err, (P[i].w - p.rho0) / p.rho0);
        }
        M[i] = meta_pack(lev, comp ? 1u : 0u, meta_age(m), val);
      }
      nact += (uint32_t)__popcll(__ballot(comp));
    }
    err = wave_max(err);
    if (lane == 0) {
      blku[b] = make_uint4(nact, 0u, 0u, (uint32_t)n << 16);
      blkerr[b] = err;
      // blocks with work join this step's active-block list, largest size
      // class first (their order there does not change any result); the
      // others report no force
      if (nact > 0u) {
        const uint32_t cls = (uint32_t)(kActClasses - 1) - min((nact - 1u) / 16u,
                                                                (uint32_t)(kActClasses - 1));
        const uint32_t part = (uint32_t)(((unsigned long long)q * kActParts) / nocc);
        const uint32_t r = cls * (uint32_t)kActParts + part;
        act[r * (uint32_t)p.act_cap + atomicAdd(&actn[r * kActnStride], 1u)] = b;
      } else {
        blkamax[b] = 0.0f;
      }
    }
  }
}


// ---------------------------------------------------------------------------
// active-block work distribution
// ---------------------------------------------------------------------------
// Exclusive prefix of the segment lengths in shared memory (pre[kActBuckets]
// = total).  Called by the whole workgroup; ends with a barrier.
__device__ inline void active_prefix(const uint32_t *__restrict__ actn, uint32_t *pre) {
  const int tid = threadIdx.x;
  if (tid < 64) {
    // one wave: each lane sums kPer consecutive segments, the lane totals
    // are scanned across the wave
    constexpr int kPer = kActBuckets / 64;
    static_assert(kActBuckets % 64 == 0, "segments come in whole waves");
    uint32_t v[kPer], s = 0u;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      s += actn[(tid * kPer + j) * kActnStride];
      v[j] = s;
    }
    uint32_t x = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t u = (uint32_t)__shfl_up((int)x, o, 64);
      if (tid >= o) x += u;
    }
    const uint32_t before = x - s;
#pragma unroll
    for (int j = 0; j < kPer; ++j) pre[tid * kPer + j + 1] = before + v[j];
    if (tid == 0) pre[0] = 0u;
  }
  __syncthreads();
}

// Block of list entry t (t < pre[kActBuckets]).
__device__ inline uint32_t active_block(const DevParams &p, const uint32_t *__restrict__ act,
                                        const uint32_t *pre, uint32_t t) {
  uint32_t lo = 0, hi = kActBuckets;  // pre[lo] <= t < pre[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (pre[mid] <= t) lo = mid; else hi = mid;
  }
  return act[lo * (uint32_t)p.act_cap + (t - pre[lo])];
}

// ---------------------------------------------------------------------------
// neighbour lists
// ---------------------------------------------------------------------------
// A particle's list holds the local candidate indices k (u16) of its
// neighbours in ascending order, which is the canonical neighbour order
// (sorted index, fluid before walls).  The search writes it, the density
// pass of the same kernel and the force pass read it.
__device__ inline uint16_t *list_row(const DevParams &p, uint16_t *list, uint32_t i) {
  return list + (size_t)i * (size_t)p.nbr_stride;
}
__device__ inline const uint16_t *list_row(const DevParams &p, const uint16_t *list, uint32_t i) {
  return list + (size_t)i * (size_t)p.nbr_stride;
}
// Entries e .. e + 3 of a row (e a multiple of four, e < the row's stride).
__device__ inline uint2 list_quad(const uint16_t *row, uint32_t e) {
  return *reinterpret_cast<const uint2 *>(row + e);
}
__device__ inline uint32_t quad_entry(const uint2 q, int j) {
  const uint32_t w = j < 2 ? q.x : q.y;
  return (j & 1) ? (w >> 16) : (w & 0xFFFFu);
}

// Walks the first n entries of a list row with kLanes lanes: lane `sub`
// takes the quads starting at e = 4 sub + 4 kLanes r for r < rounds (wave-
// uniform); use(quad, e) handles one (its entries past n are to be ignored).
// Two quads are in flight, each loaded straight into the register it is
// used from; the loads are unconditional, at most at entry `last` (the row's
// last quad), so that no lane mask stands between a load and its wait.
// With kPinned the loads are kept ahead of the work by scheduling barriers
// (a kernel under register pressure otherwise sinks them to their use).
template <uint32_t kLanes, bool kPinned = false, typename Use>
__device__ inline void walk_list(const uint16_t *row, uint32_t last, uint32_t rounds, uint32_t sub,
                                 Use &&use) {
  constexpr uint32_t kStep = 4u * kLanes;
  uint32_t e = 4u * sub;
  uint2 qa = list_quad(row, min(e, last));
  uint2 qb = list_quad(row, min(e + kStep, last));
  for (uint32_t r = 0; r < rounds; r += 2, e += 2u * kStep) {
    use(qa, e);
    qa = list_quad(row, min(e + 2u * kStep, last));
    if (kPinned) __builtin_amdgcn_sched_barrier(0);
    if (r + 1u >= rounds) break;
    use(qb, e + kStep);
    qb = list_quad(row, min(e + 3u * kStep, last));
    if (kPinned) __builtin_amdgcn_sched_barrier(0);
  }
}

// start + the number of set lanes of m below this lane.
__device__ inline uint32_t lanes_below(uint64_t m, uint32_t start) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, start));
}

__device__ inline float uniform_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ inline uint32_t uniform_u(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// ---------------------------------------------------------------------------
// neighbour search + density + Tait pressure, one workgroup per block
// ---------------------------------------------------------------------------
// The block's candidates are staged in LDS once.  Each wave takes its share
// of the block's active particles, kTestPart at a time:
//   test     the wave sweeps the candidates in chunks of 64, one candidate
//            per lane, and tests each of its particles against the chunk;
//            the hits of a particle form a lane mask, whose prefix counts
//            place them in the particle's list, so lists come out in
//            canonical order with every lane busy on every test
//   density  each particle gets kDenLanes lanes, which take its list entries
//            four at a time in turn (balanced however the hits fall) and sum
//            the kernel shape (Kahan-compensated), merged across the lanes
// The lists are built in the wave's own LDS rows and copied to memory by the
// density walk that reads them, so no pass waits on its own list stores; a
// pass with a list longer than an LDS row (or a block whose candidates are
// read from memory) builds its lists in memory instead.
constexpr int kTestPart = 4;                 // particles per wave and pass
constexpr int kDenLanes = 64 / kTestPart;    // density lanes per particle
constexpr int kLdsRow = 384;                 // entries of a wave's LDS list row
constexpr int kLdsUse = kLdsRow - 64;        // entries it holds (a chunk adds up to 64)

template <int kThreads>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(6))) k_search_density(
    DevParams p, const uint32_t *__restrict__ act, const uint32_t *__restrict__ start,
    const uint32_t *__restrict__ wstart, float4 *__restrict__ P, float4 *__restrict__ V,
    const uint32_t *__restrict__ M, float *__restrict__ pres, uint32_t *__restrict__ nnb,
    uint16_t *__restrict__ list, const float4 *__restrict__ WP, uint4 *__restrict__ blku,
    float *__restrict__ blkerr, const uint32_t *__restrict__ ids,
    const uint32_t *__restrict__ actn, DevCtrl *ctrl, DevScalars *S) {
  __shared__ Pos3 s_pos[kStageCap + 1];  // + the far slot named by list padding
  __shared__ uint2 s_lq[kThreads / 64][kTestPart][kLdsRow / 4];  // LDS list rows, in quads
  __shared__ uint32_t s_rs[18], s_ro[19], s_len[18];
  __shared__ uint16_t s_act[kCellMax];
  __shared__ uint32_t s_nact;
  __shared__ float s_err[kThreads / 64];
  __shared__ uint32_t s_inter[kThreads / 64], s_nmax[kThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  const uint32_t cap = (uint32_t)p.nbr_cap;  // neighbours; a row holds cap + 1 entries
  __shared__ uint32_t s_pre[kActBuckets + 1], s_ticket;
  if (tid == 0) s_pos[kStageCap] = Pos3{1e30f, 1e30f, 1e30f};
  // blocks with active particles are handed out one at a time (the first
  // round by workgroup index), so the workgroups finish together however
  // unevenly the work is spread
  active_prefix(actn, s_pre);
  const uint32_t nblk = s_pre[kActBuckets];
  for (uint32_t round = 0;; ++round) {
    if (tid == 0)
      s_ticket = round == 0 ? blockIdx.x : gridDim.x + atomicAdd(&ctrl->search_ticket, 1u);
    __syncthreads();
    const uint32_t q = s_ticket;
    if (q >= nblk) break;
    const uint32_t b = active_block(p, act, s_pre, q);
    const uint32_t s0 = start[b];
    const int n = min((int)(start[b + 1] - s0), kCellMax);
    if (tid == 0) s_nact = 0;
    block_ranges_shared(p, start, wstart, b, s_rs, s_ro, s_len);
    // active particles of the block (their order here does not matter)
    for (int k = tid; k < n; k += kThreads)
      if (meta_compute(M[s0 + (uint32_t)k])) s_act[atomicAdd(&s_nact, 1u)] = (uint16_t)k;
    __syncthreads();
    const uint32_t C = s_ro[18];
    const uint32_t cpad = (C + 63u) / 64u * 64u;
    const bool staged = cpad <= (uint32_t)kStageCap;
    if (staged) stage_positions<kThreads>(s_rs, s_ro, P, WP, s_pos, cpad);
    __syncthreads();
    const uint32_t nact = s_nact;
    const uint32_t self_off = s_ro[4] - s_rs[4];  // local index = sorted index + self_off
    const bool fits = C <= (uint32_t)p.cand_cap;  // list entries are 16-bit candidate indices
    if (!fits && tid == 0 && nact > 0) set_status(S, RTS_E_CAPACITY, (int32_t)ids[s0]);
    const uint32_t nch = cpad / 64u;
    // this wave's particles: slots [q_lo, q_hi) of the active list, whole
    // tiles of kTestPart (only the block's last tile can be partial)
    const uint32_t ntile = (nact + kTestPart - 1u) / kTestPart;
    const uint32_t per_wave = (ntile + (uint32_t)(kThreads / 64) - 1u) / (uint32_t)(kThreads / 64);
    const uint32_t q_lo = min((uint32_t)wave * per_wave * kTestPart, nact);
    const uint32_t q_hi = fits ? min(q_lo + per_wave * kTestPart, nact) : q_lo;
    float err = 0.0f;
    uint32_t inter = 0, nmax = 0;
    uint16_t *const lrows = reinterpret_cast<uint16_t *>(&s_lq[wave][0][0]);  // this wave's
    for (uint32_t q0 = q_lo; q0 < q_hi; q0 += kTestPart) {
      const uint32_t np = min((uint32_t)kTestPart, q_hi - q0);  // wave-uniform
      uint32_t pid[kTestPart], cnt[kTestPart];
      float px[kTestPart], py[kTestPart], pz[kTestPart];
#pragma unroll
      for (int t = 0; t < kTestPart; ++t) {
        // slots past np repeat the last particle and are never tested
        const uint32_t slot = q0 + min((uint32_t)t, np - 1u);
        pid[t] = uniform_u(s0 + (uint32_t)s_act[slot]);
        // the same in every lane, held in vector registers; a staged block
        // holds the particle among its own candidates
        if (staged) {
          const Pos3 xi = s_pos[pid[t] + self_off];
          px[t] = xi.x;
          py[t] = xi.y;
          pz[t] = xi.z;
        } else {
          const float4 xi = P[pid[t]];
          px[t] = xi.x;
          py[t] = xi.y;
          pz[t] = xi.z;
        }
        cnt[t] = 0u;
      }
      // test: lane = candidate 64 c + lane; one lane mask per particle.  The
      // particle itself is a candidate at distance 0 and enters its own list
      // (the density takes its W(0) from there; the force skips r = 0).  A
      // row holds 64 entries beyond its clamp, so the write offset is clamped
      // there and a list past the row only goes on counting.
      const auto sweep = [&](auto np_c, auto to_lds_c, auto &&candidate) {
        constexpr int kNp = decltype(np_c)::value;
        constexpr bool kLds = decltype(to_lds_c)::value;
        const auto test_chunk = [&](uint32_t c, const float4 xk) {
          const uint32_t k = 64u * c + (uint32_t)lane;
#pragma unroll
          for (int t = 0; t < kTestPart; ++t) {
            if (kNp == kTestPart ? false : (uint32_t)t >= np) break;
            const float d2 = dist2_exact(px[t], py[t], pz[t], xk.x, xk.y, xk.z);
            const bool near = d2 < p.r2f;
            const uint64_t m = __builtin_amdgcn_ballot_w64(near);
            if (kLds) {
              const uint32_t base = (uint32_t)t * kLdsRow + min(cnt[t], (uint32_t)kLdsUse);
              if (near) lrows[base + lanes_below(m, 0u)] = (uint16_t)k;
            } else {
              const uint32_t off = 2u * min(cnt[t], cap + 1u);  // bytes, wave-uniform
              if (near)
                *reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(list_row(p, list, pid[t])) +
                                              off + 2u * lanes_below(m, 0u)) = (uint16_t)k;
            }
            cnt[t] += (uint32_t)__popcll(m);
          }
        };
        // two chunks in flight, each loaded into the register it is tested
        // from
        float4 xa = candidate((uint32_t)lane);
        float4 xb = candidate(64u + (uint32_t)lane);  // not tested when nch == 1
        for (uint32_t c = 0; c < nch; c += 2u) {
          test_chunk(c, xa);
          if (c + 2u < nch) xa = candidate(64u * (c + 2u) + (uint32_t)lane);
          if (c + 1u >= nch) break;
          test_chunk(c + 1u, xb);
          if (c + 3u < nch) xb = candidate(64u * (c + 3u) + (uint32_t)lane);
        }
      };
      using Full = std::integral_constant<int, kTestPart>;
      using Part = std::integral_constant<int, 0>;
      using Lds = std::true_type;
      using Mem = std::false_type;
      const auto staged_pos = [&](uint32_t k) {  // slots from C to cpad are far away
        const Pos3 q = s_pos[k];
        return make_float4(q.x, q.y, q.z, 0.0f);
      };
      const auto memory_pos = [&](uint32_t k) {
        float4 xk = make_float4(1e30f, 1e30f, 1e30f, 0.0f);
        if (k < C) {
          bool wall;
          const uint32_t j = local_to_global(s_rs, s_ro, k, wall);
          xk = wall ? WP[j] : P[j];
        }
        return xk;
      };
      bool in_lds = staged;
      if (staged) {
        // one loop per candidate source, so that this loop waits on
        // shared-memory loads only
        if (np == kTestPart) sweep(Full{}, Lds{}, staged_pos); else sweep(Part{}, Lds{}, staged_pos);
#pragma unroll
        for (int t = 0; t < kTestPart; ++t) in_lds = in_lds && cnt[t] <= (uint32_t)kLdsUse;
      }
      if (!in_lds) {
        // a list longer than an LDS row, or candidates from memory: the
        // lists are built in memory (rare)
#pragma unroll
        for (int t = 0; t < kTestPart; ++t) cnt[t] = 0u;
        if (staged) sweep(Part{}, Mem{}, staged_pos); else sweep(Part{}, Mem{}, memory_pos);
      }
      // a particle whose own test failed (a non-finite position) gets itself
      // as its one entry, so that every entry names a real candidate
      uint32_t most = 0;  // longest list of the pass, wave-uniform
#pragma unroll
      for (int t = 0; t < kTestPart; ++t) {
        if ((uint32_t)t >= np) break;
        if (cnt[t] == 0u) {
          const uint16_t self = (uint16_t)(pid[t] + self_off);
          if (lane == 0) {
            if (in_lds) lrows[t * kLdsRow] = self; else list_row(p, list, pid[t])[0] = self;
          }
          cnt[t] = 1u;
        }
        if (lane == 0 && cnt[t] > cap + 1u) set_status(S, RTS_E_CAPACITY, (int32_t)ids[pid[t]]);
        cnt[t] = min(cnt[t], cap + 1u);
        most = max(most, cnt[t]);
      }
      const uint32_t span = (most + 4u * kDenLanes - 1u) / (4u * kDenLanes) * (4u * kDenLanes);
      if (staged) {
        // entries from a list's end to the pass's span name the far slot,
        // whose kernel value is exactly zero: the density walk then needs no
        // per-entry bounds
#pragma unroll
        for (int t = 0; t < kTestPart; ++t) {
          if ((uint32_t)t >= np) break;
          if (in_lds) {
            for (uint32_t e = cnt[t] + (uint32_t)lane; e < span; e += 64u)
              lrows[t * kLdsRow + e] = (uint16_t)kStageCap;
          } else {
            uint16_t *row = list_row(p, list, pid[t]);
            for (uint32_t e = cnt[t] + (uint32_t)lane; e < span; e += 64u) row[e] = (uint16_t)kStageCap;
          }
        }
      }
      // the entries become visible to the wave's other lanes: shared memory
      // in order within the wave, memory through a fence
      if (in_lds) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      }
      // density: lanes [kDenLanes g, kDenLanes (g + 1)) take particle g
      const uint32_t g = (uint32_t)lane / kDenLanes, sub = (uint32_t)lane % kDenLanes;
      uint32_t i = pid[0], ng = cnt[0];
      float xg = px[0], yg = py[0], zg = pz[0];
#pragma unroll
      for (int t = 1; t < kTestPart; ++t) {
        if ((uint32_t)t == g) {
          i = pid[t];
          ng = cnt[t];
          xg = px[t];
          yg = py[t];
          zg = pz[t];
        }
      }
      const bool live = g < np;
      if (!live) ng = 0u;
      uint16_t *row = list_row(p, list, i);
      float sum = 0.0f, comp = 0.0f;
      const auto add = [&](const float4 qj) {
        const float d2 = dist2_exact(xg, yg, zg, qj.x, qj.y, qj.z);
        const float wk = w_shape(__builtin_amdgcn_sqrtf(d2) * p.inv_h);
        const float y2 = wk - comp;
        const float tt = sum + y2;
        comp = (tt - sum) - y2;
        sum = tt;
      };
      const auto add_quad = [&](const uint2 qd) {
        float4 v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = staged_pos(quad_entry(qd, j));
#pragma unroll
        for (int j = 0; j < 4; ++j) add(v[j]);
      };
      const uint32_t rounds = span / (4u * kDenLanes);
      const uint32_t last = (uint32_t)p.nbr_stride - 4u;
      if (in_lds) {
        // quads of the wave's LDS row, copied to the memory row on the way
        // (a live particle's row; lanes past np walk a repeated row)
        const uint2 *lq = &s_lq[wave][min(g, np - 1u)][0];
        for (uint32_t r = 0; r < rounds; ++r) {
          const uint32_t e = 4u * sub + 4u * kDenLanes * r;
          const uint2 qd = lq[e / 4u];
          if (live) *reinterpret_cast<uint2 *>(row + e) = qd;
          add_quad(qd);
        }
      } else if (staged) {
        walk_list<kDenLanes>(row, last, rounds, sub, [&](const uint2 qd, uint32_t) { add_quad(qd); });
      } else {
        walk_list<kDenLanes>(row, last, rounds, sub, [&](const uint2 qd, uint32_t e) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (e + (uint32_t)j >= ng) break;
            bool wall;
            const uint32_t jj = local_to_global(s_rs, s_ro, quad_entry(qd, j), wall);
            add(wall ? WP[jj] : P[jj]);
          }
        });
      }
      // merge the particle's lanes (adjacent)
#pragma unroll
      for (int o = 1; o < kDenLanes; o <<= 1) {
        const float s2 = __shfl_xor(sum, o, 64), c2 = __shfl_xor(comp, o, 64);
        kahan_merge(sum, comp, s2, c2);
      }
      if (live && sub == 0) {
        // rho/rho0 - 1 = (m sigma / rho0) (sum - C) with C = rho0/(m sigma),
        // sum = sum of the kernel shape over the list (the particle's own
        // W(0) = 1 included), carried as sum - comp; the difference is
        // formed before any rounding to rho.
        const float dev = p.kms * ((sum - p.cs_hi) - (comp + p.cs_lo));
        const float rho = p.rho0 + p.rho0 * dev;
        const float pr = tait_from_dev(p, dev);
        reinterpret_cast<float *>(&P[i])[3] = rho;
        reinterpret_cast<float *>(&V[i])[3] = pr / (rho * rho);
        pres[i] = pr;
        nnb[i] = ng - 1u;  // neighbours, the particle itself not counted
        err = fmaxf(err, dev);
        inter += ng - 1u;
        nmax = max(nmax, ng - 1u);
      }
      // the next pass rewrites the wave's LDS rows
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    err = wave_max(err);
    inter = wave_sum_u32(inter);
    nmax = wave_max_u32(nmax);
    if (lane == 0) {
      s_err[wave] = err;
      s_inter[wave] = inter;
      s_nmax[wave] = nmax;
    }
    __syncthreads();
    if (tid == 0) {
      float e = blkerr[b];  // inactive particles, from the flags pass
      uint32_t it = 0, nm = 0;
      for (int w = 0; w < kThreads / 64; ++w) {
        e = fmaxf(e, s_err[w]);
        it += s_inter[w];
        nm = max(nm, s_nmax[w]);
      }
      blku[b] = make_uint4(nact, it, nact * C, nm | ((uint32_t)n << 16));
      blkerr[b] = e;
    }
    __syncthreads();  // shared memory is reused by the next block
  }
}

// ---------------------------------------------------------------------------
// forces, one workgroup per block
// ---------------------------------------------------------------------------
// 4 or 8 lanes per active particle (a launch-shape choice) take its list
// entries four at a time in turn; the candidates' position, density,
// velocity and p / rho^2 are staged in LDS.

// Velocity slot of a wall candidate: at rest, and g . x in place of p / rho^2.
__device__ inline float4 wall_slot(const DevParams &p, const float4 q) {
  return make_float4(0.0f, 0.0f, 0.0f, p.g[0] * q.x + p.g[1] * q.y + p.g[2] * q.z);
}

// A particle's acceleration is summed in a fixed decomposition that does not
// depend on how many lanes share the particle: its list's quads go round-robin
// to kVirt partial sums (quad q to sum q mod kVirt, each in list order), and
// the partial sums are folded pairwise at distances kVirt/2, ..., 2, 1.  With
// kLanes lanes a lane holds kVirt / kLanes of them (lane s the sums s,
// s + kLanes, ...); the folds at distances of at least kLanes are within a
// lane, the rest across lanes.  A float sum of two terms does not depend on
// their order, so every lane count gives the same bits.  Eight sums: at
// eight lanes a lane holds one (a 16-way split costs the eight-lane shape
// the registers of a second, and spills).
constexpr int kVirt = 8;

// Walks a list row like walk_list, kDepth quads in flight; use(quad, e, d)
// gets the quad's round phase d = round mod kDepth as a compile-time constant
// (std::integral_constant), so per-phase partial sums stay in registers.
template <uint32_t kLanes, uint32_t kDepth, typename Use, uint32_t... D>
__device__ inline void walk_list_phased_(const uint16_t *row, uint32_t last, uint32_t rounds,
                                         uint32_t sub, Use &&use,
                                         std::integer_sequence<uint32_t, D...>) {
  constexpr uint32_t kStep = 4u * kLanes;
  uint32_t e = 4u * sub;
  uint2 q[kDepth];
#pragma unroll
  for (uint32_t d = 0; d < kDepth; ++d) q[d] = list_quad(row, min(e + d * kStep, last));
  for (uint32_t r = 0; r < rounds; r += kDepth, e += kDepth * kStep) {
    (
        [&] {
          if (r + D < rounds) {
            use(q[D], e + D * kStep, std::integral_constant<uint32_t, D>{});
            q[D] = list_quad(row, min(e + (kDepth + D) * kStep, last));
            // keeps the load ahead of its use (the kernel's register
            // pressure would otherwise sink it there)
            __builtin_amdgcn_sched_barrier(0);
          }
        }(),
        ...);
  }
}
template <uint32_t kLanes, uint32_t kDepth, typename Use>
__device__ inline void walk_list_phased(const uint16_t *row, uint32_t last, uint32_t rounds,
                                        uint32_t sub, Use &&use) {
  walk_list_phased_<kLanes, kDepth>(row, last, rounds, sub, use,
                                    std::make_integer_sequence<uint32_t, kDepth>{});
}

template <int kLanes>
__global__ void __launch_bounds__(kForceThreads) __attribute__((amdgpu_waves_per_eu(4))) k_force(
    DevParams p, const uint32_t *__restrict__ act, const uint32_t *__restrict__ start,
    const uint32_t *__restrict__ wstart, const float4 *__restrict__ P,
    const float4 *__restrict__ V, const uint32_t *__restrict__ M,
    const uint32_t *__restrict__ nnb, const uint16_t *__restrict__ list,
    const float4 *__restrict__ WP, float4 *__restrict__ anew, float *__restrict__ blkamax,
    const uint32_t *__restrict__ actn, DevCtrl *ctrl) {
  static_assert(kLanes == 4 || kLanes == 8, "lanes per particle divide kVirt");
  constexpr int kAcc = kVirt / kLanes;                  // partial sums per lane
  constexpr uint32_t kDepth = kAcc > 2 ? (uint32_t)kAcc : 2u;  // quads in flight
  constexpr int kPerPass = kForceThreads / kLanes;      // particles per workgroup pass
  __shared__ float4 s_p[kForceCap];
  __shared__ float4 s_v[kForceCap];
  __shared__ uint32_t s_rs[18], s_ro[19], s_len[18];
  __shared__ uint16_t s_act[kCellMax];
  __shared__ uint32_t s_nact;
  __shared__ float s_amax[kForceThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t sub = (uint32_t)(tid & (kLanes - 1));
  const uint32_t cap = (uint32_t)p.nbr_cap;
  // -m grad W(x_ij) = f x_ij with f = -m (sigma / h) w'(q) / r, q = r / h:
  // f = fA + fB q for q < 1, f = fC (2 - q)^2 / r for 1 <= q < 2
  const float mcoefg = -p.mass * p.sigma * p.inv_h;
  const float fA = -3.0f * mcoefg * p.inv_h, fB = 2.25f * mcoefg * p.inv_h, fC = -0.75f * mcoefg;
  __shared__ uint32_t s_pre[kActBuckets + 1], s_ticket;
  active_prefix(actn, s_pre);
  const uint32_t nblk = s_pre[kActBuckets];
  for (uint32_t round = 0;; ++round) {
    if (tid == 0)
      s_ticket = round == 0 ? blockIdx.x : gridDim.x + atomicAdd(&ctrl->force_ticket, 1u);
    __syncthreads();
    const uint32_t q = s_ticket;
    if (q >= nblk) break;
    const uint32_t b = active_block(p, act, s_pre, q);
    const uint32_t s0 = start[b];
    const int n = min((int)(start[b + 1] - s0), kCellMax);
    if (tid == 0) s_nact = 0;
    block_ranges_shared(p, start, wstart, b, s_rs, s_ro, s_len);
    for (int k = tid; k < n; k += kForceThreads)
      if (meta_compute(M[s0 + (uint32_t)k])) s_act[atomicAdd(&s_nact, 1u)] = (uint16_t)k;
    __syncthreads();
    const uint32_t C = s_ro[18], Cf = s_ro[9];
    const bool staged = C <= (uint32_t)kForceCap;
    if (staged) {
      // positions (walls included), then velocities: the four loads of a
      // phase are issued before its shared-memory writes.  Named registers,
      // not an array, so nothing lands in private memory.
      static_assert(kForceCap == 4 * kForceThreads, "staging assumes four slots per thread");
      const uint32_t k0 = (uint32_t)tid, k1 = k0 + kForceThreads, k2 = k1 + kForceThreads,
                     k3 = k2 + kForceThreads;
      uint32_t j0, j1, j2, j3;
      const float4 b0 = stage_load(s_rs, s_ro, P, WP, k0, C, j0);
      const float4 b1 = stage_load(s_rs, s_ro, P, WP, k1, C, j1);
      const float4 b2 = stage_load(s_rs, s_ro, P, WP, k2, C, j2);
      const float4 b3 = stage_load(s_rs, s_ro, P, WP, k3, C, j3);
      if (k0 < C) s_p[k0] = b0;
      if (k1 < C) s_p[k1] = b1;
      if (k2 < C) s_p[k2] = b2;
      if (k3 < C) s_p[k3] = b3;
      const float4 u0 = j0 != kNoFluid ? V[j0] : wall_slot(p, b0);
      const float4 u1 = j1 != kNoFluid ? V[j1] : wall_slot(p, b1);
      const float4 u2 = j2 != kNoFluid ? V[j2] : wall_slot(p, b2);
      const float4 u3 = j3 != kNoFluid ? V[j3] : wall_slot(p, b3);
      if (k0 < C) s_v[k0] = u0;
      if (k1 < C) s_v[k1] = u1;
      if (k2 < C) s_v[k2] = u2;
      if (k3 < C) s_v[k3] = u3;
    }
    __syncthreads();
    const uint32_t nact = s_nact;
    float a2max = 0.0f;
    for (uint32_t c0 = 0; c0 < nact && C <= (uint32_t)p.cand_cap; c0 += kPerPass) {
      if (c0 + (uint32_t)(wave * (64 / kLanes)) >= nact) break;
      const uint32_t slot = c0 + (uint32_t)(tid / kLanes);
      const bool live = slot < nact;
      const uint32_t i = s0 + (live ? (uint32_t)s_act[slot] : 0u);
      const float4 pi = P[i], vi = V[i];
      const float rhoi = pi.w, pri = vi.w;
      const float inv_rhoi = __builtin_amdgcn_rcpf(rhoi);
      float ax[kAcc], ay[kAcc], az[kAcc];
#pragma unroll
      for (int k = 0; k < kAcc; ++k) ax[k] = ay[k] = az[k] = 0.0f;
      // a static wall particle is at rest and mirrors the density and the
      // pressure of the fluid particle, plus the hydrostatic difference
      // g . (x_j - x_i), clamped at zero; uj.w of a wall holds g . x_j
      const float gxi = p.g[0] * pi.x + p.g[1] * pi.y + p.g[2] * pi.z;
      auto pair = [&](const float4 qj, const float4 uj, bool wall, bool valid, auto kc) {
        constexpr int k = (int)decltype(kc)::value;
        const float rhoj = wall ? rhoi : qj.w;
        const float prj = wall ? fmaxf(pri + (uj.w - gxi) * inv_rhoi, 0.0f) : uj.w;
        const float dx = pi.x - qj.x, dy = pi.y - qj.y, dz = pi.z - qj.z;
        const float r2 = dx * dx + dy * dy + dz * dz;
        const float rinv = __builtin_amdgcn_rsqf(r2);
        const float q = r2 * rinv * p.inv_h;
        const float t = fmaxf(2.0f - q, 0.0f);
        const float f1 = fmaf(fB, q, fA), f2 = fC * t * t * rinv;
        const float f = __builtin_unpredictable(q < 1.0f) ? f1 : f2;  // -m gradW = f x_ij
        const float vx = (vi.x - uj.x) * dx + (vi.y - uj.y) * dy + (vi.z - uj.z) * dz;
        // artificial viscosity -nu vx / (r^2 + eps h^2), nu = 2 alpha h c0 / (rho_i + rho_j)
        const float visc = -p.visc_num * vx *
                           __builtin_amdgcn_rcpf((rhoi + rhoj) * (r2 + p.visc_eps_h2));
        const float coef = pri + prj + (vx < 0.0f ? visc : 0.0f);
        const float sc = valid && r2 > 0.0f ? coef * f : 0.0f;
        ax[k] += sc * dx;
        ay[k] += sc * dy;
        az[k] += sc * dz;
      };
      // list entries: the neighbours and the particle itself (r = 0, skipped)
      const uint32_t cnt = live ? min(nnb[i], cap) + 1u : 0u;
      const uint16_t *row = list_row(p, list, i);
      // rounds of 4 kLanes entries, as many as the wave's longest list needs
      const uint32_t most = wave_max_u32(cnt);
      const uint32_t rounds = (most + 4u * kLanes - 1u) / (4u * kLanes);
      const uint32_t last = (uint32_t)p.nbr_stride - 4u;
      if (staged) {
        walk_list_phased<kLanes, kDepth>(row, last, rounds, sub,
                                         [&](const uint2 qd, uint32_t e, auto dc) {
          // this round's partial sum
          const std::integral_constant<int, (int)(decltype(dc)::value % kAcc)> k{};
          uint32_t kk[4];
          bool ok[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            ok[j] = e + (uint32_t)j < cnt;
            kk[j] = ok[j] ? quad_entry(qd, j) : 0u;
          }
          float4 qa[4], ua[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            qa[j] = s_p[kk[j]];
            ua[j] = s_v[kk[j]];
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) pair(qa[j], ua[j], kk[j] >= Cf, ok[j], k);
        });
      } else {
        walk_list_phased<kLanes, kDepth>(row, last, rounds, sub,
                                         [&](const uint2 qd, uint32_t e, auto dc) {
          const std::integral_constant<int, (int)(decltype(dc)::value % kAcc)> k{};
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (e + (uint32_t)j >= cnt) break;
            const uint32_t kq = quad_entry(qd, j);
            bool wall;
            const uint32_t jj = local_to_global(s_rs, s_ro, kq, wall);
            const float4 qj = wall ? WP[jj] : P[jj];
            pair(qj, wall ? wall_slot(p, qj) : V[jj], wall, true, k);
          }
        });
      }
      // fold the kVirt partial sums at distances kVirt/2, ..., 1: within the
      // lane while the distance is at least kLanes, then across lanes
#pragma unroll
      for (int o = kVirt / 2; o >= 1; o >>= 1) {
        if (o >= kLanes) {
#pragma unroll
          for (int k = 0; k < o / kLanes; ++k) {
            ax[k] = ax[k] + ax[k + o / kLanes];
            ay[k] = ay[k] + ay[k + o / kLanes];
            az[k] = az[k] + az[k + o / kLanes];
          }
        } else {
          ax[0] += __shfl_xor(ax[0], o, 64);
          ay[0] += __shfl_xor(ay[0], o, 64);
          az[0] += __shfl_xor(az[0], o, 64);
        }
      }
      if (live && sub == 0) {
        const float gx = ax[0] + p.g[0], gy = ay[0] + p.g[1], gz = az[0] + p.g[2];
        anew[i] = make_float4(gx, gy, gz, 0.0f);
        a2max = fmaxf(a2max, gx * gx + gy * gy + gz * gz);
      }
    }
    a2max = wave_max(a2max);
    if (lane == 0) s_amax[wave] = a2max;
    __syncthreads();
    if (tid == 0) {
      float m = 0.0f;
      for (int w2 = 0; w2 < kForceThreads / 64; ++w2) m = fmaxf(m, s_amax[w2]);
      blkamax[b] = m;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// per-step statistics and the step length (kStatBlocks workgroups; the last
// one to finish folds the partials)
// ---------------------------------------------------------------------------
__device__ inline void part_add(StatPart &t, const StatPart &u) {
  t.act += u.act;
  t.inter += u.inter;
  t.cand += u.cand;
  t.nmax = max(t.nmax, u.nmax);
  t.err = fmaxf(t.err, u.err);
  t.amax2 = fmaxf(t.amax2, u.amax2);
  for (int k = 0; k < kMaxLevels; ++k) t.hist[k] += u.hist[k];
}

// Workgroup `wg` of `nwg` (256 threads each); every one of the nwg must run it.
__device__ inline void step_stats_body(const DevParams &p, const uint32_t *__restrict__ occ,
                                       const uint4 *__restrict__ blku,
                                       const float *__restrict__ blkerr,
                                       const float *__restrict__ blkamax,
                                       const uint8_t *__restrict__ lvl,
                                       StatPart *__restrict__ part, DevCtrl *ctrl, DevScalars *S,
                                       uint32_t wg, uint32_t nwg) {
  __shared__ StatPart s_w[4];
  __shared__ uint32_t s_last;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t nocc = S->n_occ;
  StatPart t = {};
  for (uint32_t q = wg * 256u + (uint32_t)tid; q < nocc; q += nwg * 256u) {
    const uint32_t b = occ[q];
    const uint4 u = blku[b];
    t.act += u.x;
    t.inter += u.y;
    t.cand += u.z;
    t.nmax = max(t.nmax, u.w & 0xFFFFu);
    t.err = fmaxf(t.err, blkerr[b]);
    t.amax2 = fmaxf(t.amax2, blkamax[b]);
    const uint32_t l = lvl[b];
#pragma unroll
    for (int k = 0; k < kMaxLevels; ++k)
      t.hist[k] += (l == (uint32_t)k) ? (int32_t)(u.w >> 16) : 0;
  }
  for (int o = 32; o > 0; o >>= 1) {
    t.act += __shfl_xor(t.act, o, 64);
    t.inter += __shfl_xor(t.inter, o, 64);
    t.cand += __shfl_xor(t.cand, o, 64);
    t.nmax = max(t.nmax, (uint32_t)__shfl_xor((int)t.nmax, o, 64));
    t.err = fmaxf(t.err, __shfl_xor(t.err, o, 64));
    t.amax2 = fmaxf(t.amax2, __shfl_xor(t.amax2, o, 64));
#pragma unroll
    for (int k = 0; k < kMaxLevels; ++k) t.hist[k] += __shfl_xor(t.hist[k], o, 64);
  }
  if (lane == 0) s_w[wave] = t;
  __syncthreads();
  if (tid == 0) {
    StatPart w = s_w[0];
    for (int k = 1; k < 4; ++k) part_add(w, s_w[k]);
    part[wg] = w;
    __threadfence();
    s_last = atomicAdd(&ctrl->stats_ticket, 1u) == nwg - 1u ? 1u : 0u;
  }
  __syncthreads();
  if (!s_last || wave != 0) return;
  __threadfence();
  // one wave folds the partials: lane g reads partial g
  StatPart a = {};
  for (unsigned g = (unsigned)lane; g < nwg; g += 64) part_add(a, part[g]);
  for (int o = 32; o > 0; o >>= 1) {
    a.act += __shfl_xor(a.act, o, 64);
    a.inter += __shfl_xor(a.inter, o, 64);
    a.cand += __shfl_xor(a.cand, o, 64);
    a.nmax = max(a.nmax, (uint32_t)__shfl_xor((int)a.nmax, o, 64));
    a.err = fmaxf(a.err, __shfl_xor(a.err, o, 64));
    a.amax2 = fmaxf(a.amax2, __shfl_xor(a.amax2, o, 64));
#pragma unroll
    for (int k = 0; k < kMaxLevels; ++k) a.hist[k] += __shfl_xor(a.hist[k], o, 64);
  }
  if (lane != 0) return;
  S->n_act = (uint32_t)a.act;
  S->inter_last = a.inter;
  S->cand_last = a.cand;
  S->active_total += a.act;
  S->inter_total += a.inter;
  S->cand_total += a.cand;
  S->nbr_max = max(S->nbr_max, a.nmax);
  S->err_last = a.err;
  S->err_run = fmaxf(S->err_run, a.err);
  S->amax2 = a.amax2;
  for (int k = 0; k < kMaxLevels; ++k) S->hist[k] = a.hist[k];
  // the step length: fixed, or the adaptive comparator's
  double dtd = p.dt_base;
  if (p.mode == RTS_MODE_GLOBAL_ADAPTIVE) {
    dtd = p.dt_cfl;
    if (a.amax2 > 0.0f) {
      const double df = sqrt(p.lf2r / sqrt((double)a.amax2));
      if (df < dtd) dtd = df;
    }
  }
  S->dt_next = dtd;
  S->time += dtd;
  S->step += 1;
  ctrl->stats_ticket = 0u;
}

__global__ void __launch_bounds__(256) k_step_stats(DevParams p, const uint32_t *__restrict__ occ,
                                                   const uint4 *__restrict__ blku,
                                                   const float *__restrict__ blkerr,
                                                   const float *__restrict__ blkamax,
                                                   const uint8_t *__restrict__ lvl,
                                                   StatPart *__restrict__ part, DevCtrl *ctrl,
                                                   DevScalars *S) {
  step_stats_body(p, occ, blku, blkerr, blkamax, lvl, part, ctrl, S, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// corrector (active) + predictor (all)
// ---------------------------------------------------------------------------
// Particle i with step dt; dt_prev is the last step's length (global
// adaptive comparator only).
__device__ inline float4 correct_predict_one(const DevParams &p, float4 *__restrict__ P,
                                           float4 *__restrict__ V, float4 *__restrict__ A,
                                           uint32_t *__restrict__ M,
                                           const float4 *__restrict__ anew, int i, float dt,
                                           float dt_prev) {
  float4 x = P[i], v = V[i], a = A[i];
  const uint32_t m = M[i];
  uint32_t age = meta_age(m);
  if (meta_compute(m)) {
    const float4 an = anew[i];
    if (p.serna_correct) {
      const float dtau = p.mode == RTS_MODE_GLOBAL_ADAPTIVE ? dt_prev : (float)age * p.dt_base;
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
  return x;
}

__global__ void __launch_bounds__(256) k_correct_predict(DevParams p, float4 *__restrict__ P,
                                                        float4 *__restrict__ V,
                                                        float4 *__restrict__ A,
                                                        uint32_t *__restrict__ M,
                                                        const float4 *__restrict__ anew,
                                                        const DevScalars *__restrict__ S) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  (void)correct_predict_one(p, P, V, A, M, anew, i, (float)S->dt_next, (float)S->dt_prev);
}

// Fixed base step (RTS, global fixed): the corrector-predictor does not wait
// for the statistics, so one launch carries both; it also bins the predicted
// positions for the next step's sort (keys, histogram, domain check) and
// resets that step's counters, so the next step starts with its scan.
// Workgroups below kStatBlocks also take their share of the statistics.
__global__ void __launch_bounds__(256) k_stats_correct_predict(
    DevParams p, const uint32_t *__restrict__ occ, const uint4 *__restrict__ blku,
    const float *__restrict__ blkerr, const float *__restrict__ blkamax,
    const uint8_t *__restrict__ lvl, StatPart *__restrict__ part, DevCtrl *ctrl, DevScalars *S,
    float4 *__restrict__ P, float4 *__restrict__ V, float4 *__restrict__ A,
    uint32_t *__restrict__ M, const float4 *__restrict__ anew, const uint32_t *__restrict__ ids,
    uint32_t *__restrict__ keyold, uint32_t *__restrict__ rank, uint32_t *__restrict__ count,
    uint32_t *__restrict__ actn) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = i < p.n;
  float4 x = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if (live) x = correct_predict_one(p, P, V, A, M, anew, i, p.dt_base, p.dt_base);
  bin_particle(p, i, live, x, ids, keyold, rank, count, S);
  step_controls_reset(i, ctrl, actn);
  if (blockIdx.x < (unsigned)kStatBlocks)
    step_stats_body(p, occ, blku, blkerr, blkamax, lvl, part, ctrl, S, blockIdx.x, kStatBlocks);
}

// ---------------------------------------------------------------------------
// state in / out, walls, debug views
// ---------------------------------------------------------------------------
__global__ void k_set_state(DevParams p, const float *__restrict__ pos,
                            const float *__restrict__ vel, float4 *P, float4 *V, float4 *A,
                            uint32_t *M, uint32_t *ID, float *pres) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  const size_t n = (size_t)p.n;
  P[i] = make_float4(pos[i], pos[n + i], pos[2 * n + i], p.rho0);
  V[i] = vel ? make_float4(vel[i], vel[n + i], vel[2 * n + i], 0.0f)
             : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  A[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  M[i] = meta_pack(0xFu, 0u, 0u, 0);
  ID[i] = (uint32_t)i;
  pres[i] = 0.0f;
}

// External impulse: the caller's velocity change (planes, caller order) is
// added to each particle's velocity; levels, validity, ages and stored
// accelerations stay as they are, so the next step's block maxima see the
// change and pre-empt the particles whose block needs a smaller step.
__global__ void k_add_velocity(DevParams p, const float *__restrict__ dv, const uint32_t *ID,
                               float4 *V) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  const size_t n = (size_t)p.n;
  const uint32_t c = ID[i];
  float4 v = V[i];
  v.x += dv[c];
  v.y += dv[n + c];
  v.z += dv[2 * n + c];
  V[i] = v;
}

__global__ void k_get_state(DevParams p, const float4 *P, const float4 *V, const float4 *A,
                            const uint32_t *M, const uint32_t *ID, uint32_t lo, uint32_t cnt,
                            float *pos, float *vel, float *acc, float *rho, float *po,
                            uint8_t *level) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  // caller indices [lo, lo + cnt) go to slots [0, cnt) of the planes
  const uint32_t c = ID[i] - lo;
  if (c >= cnt) return;
  const size_t n = (size_t)cnt;
  const float4 x = P[i];
  if (pos) { pos[c] = x.x; pos[n + c] = x.y; pos[2 * n + c] = x.z; }
  if (vel) { const float4 v = V[i]; vel[c] = v.x; vel[n + c] = v.y; vel[2 * n + c] = v.z; }
  if (acc) { const float4 a = A[i]; acc[c] = a.x; acc[n + c] = a.y; acc[2 * n + c] = a.z; }
  if (rho) rho[c] = x.w;
  if (po) po[c] = V[i].w * x.w * x.w;  // V.w holds p / rho^2
  if (level) level[c] = (uint8_t)meta_level(M[i]);
}

// SplitMix64: output number `idx` (0-based) of the stream started at `seed`.
__device__ inline unsigned long long splitmix64(unsigned long long seed,
                                                unsigned long long idx) {
  unsigned long long z = seed + (idx + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Column of counts[0] x counts[1] x counts[2] lattice sites (x fastest) at
// corner + (i + 1/2) spacing, each axis offset by jitter (2u - 1) with u the
// top 24 bits of SplitMix64 draw 3 (first_draw + k) + axis, scaled by 2^-24.
// Double precision, every operation rounded on its own (no fused
// multiply-add), then rounded once to float.
__global__ void k_init_lattice(DevParams p, uint32_t first, uint32_t cnt, LatticeSpec L,
                               float4 *P, float4 *V, float4 *A, uint32_t *M, uint32_t *ID,
                               float *pres) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= cnt) return;
  const uint32_t ix = k % (uint32_t)L.counts[0];
  const uint32_t iy = (k / (uint32_t)L.counts[0]) % (uint32_t)L.counts[1];
  const uint32_t iz = k / ((uint32_t)L.counts[0] * (uint32_t)L.counts[1]);
  const uint32_t idx[3] = {ix, iy, iz};
  float x[3];
  for (int a = 0; a < 3; ++a) {
    double q = __dadd_rn(L.corner[a], __dmul_rn((double)idx[a] + 0.5, L.spacing));
    if (L.jitter != 0.0) {
      const unsigned long long draw = 3ull * (L.first_draw + k) + (unsigned long long)a;
      const double u = (double)(splitmix64(L.seed, draw) >> 40) * 0x1p-24;
      q = __dadd_rn(q, __dmul_rn(L.jitter, 2.0 * u - 1.0));
    }
    x[a] = (float)q;
  }
  const uint32_t i = first + k;
  P[i] = make_float4(x[0], x[1], x[2], p.rho0);
  V[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  A[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  M[i] = meta_pack(0xFu, 0u, 0u, 0);
  ID[i] = i;
  pres[i] = 0.0f;
}

// Scene of caller index c: the largest s with off[s] <= c.
__device__ inline uint32_t scene_of(const uint32_t *__restrict__ off, int ns, uint32_t c) {
  uint32_t lo = 0, hi = (uint32_t)ns;   // off[lo] <= c < off[hi]
  while (hi - lo > 1u) {
    const uint32_t mid = (lo + hi) >> 1;
    if (off[mid] <= c) lo = mid; else hi = mid;
  }
  return lo;
}

// Per-scene counters of the last step from the particles' flags, levels,
// neighbour counts and stored densities.
__global__ void k_scene_stats(DevParams p, const float4 *__restrict__ P,
                              const uint32_t *__restrict__ M, const uint32_t *__restrict__ ID,
                              const uint32_t *__restrict__ nnb, const uint32_t *__restrict__ off,
                              SceneStat *st) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  const uint32_t s = scene_of(off, p.n_scenes, ID[i]);
  const uint32_t m = M[i];
  if (meta_compute(m)) {
    atomicAdd(&st[s].act, 1u);
    atomicAdd(&st[s].inter, (unsigned long long)nnb[i]);
  }
  const float e = fmaxf((P[i].w - p.rho0) / p.rho0, 0.0f);
  atomicMax(&st[s].err_bits, __float_as_uint(e));
  const uint32_t lev = meta_level(m);
  if (lev < (uint32_t)kMaxLevels) atomicAdd(&st[s].hist[lev], 1);
}

// Canonical global neighbour lists of the last step's active particles:
// out[i * kDebugRow + e] = fluid sorted index, or wall sorted index | bit 31.
__global__ void k_debug_lists(DevParams p, const uint32_t *key, const uint32_t *start,
                              const uint32_t *wstart, const uint32_t *M, const uint32_t *nnb,
                              const uint16_t *list, uint32_t *out, uint32_t *out_n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  if (!meta_compute(M[i])) {
    out_n[i] = 0;
    return;
  }
  uint32_t rs[18], ro[19];
  const int3 c = coords_of(p, key[i]);
  uint32_t acc = 0;
  for (int r = 0; r < 18; ++r) {
    uint32_t len;
    row_range(p, start, wstart, c, r, rs[r], len);
    ro[r] = acc;
    acc += len;
  }
  ro[18] = acc;
  const uint16_t *row = list + (size_t)i * (size_t)p.nbr_stride;
  const uint32_t cnt = min(nnb[i], (uint32_t)p.nbr_cap) + 1u;  // the particle itself included
  const uint32_t self = (uint32_t)i - rs[4] + ro[4];
  uint32_t o = 0;
  for (uint32_t e = 0; e < cnt; ++e) {
    const uint32_t k = row[e];
    if (k == self) continue;
    bool wall;
    const uint32_t j = local_to_global(rs, ro, k, wall);
    if (o < (uint32_t)RTS_DEBUG_NBR_ROW) out[(size_t)i * RTS_DEBUG_NBR_ROW + o] = wall ? (j | kWallBit) : j;
    ++o;
  }
  out_n[i] = o;
}

__global__ void k_wall_keys(DevParams p, const float *__restrict__ pos, uint32_t *wkey,
                            uint32_t *wrank, uint32_t *count) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= p.nw) return;
  const size_t n = (size_t)p.nw;
  const uint32_t k = key_of(p, block_of(p, pos[w], pos[n + w], pos[2 * n + w]));
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
  const size_t nw = (size_t)p.nw;
  for (int k = lane; k < n; k += 64) {
    const uint32_t src = canon ? s_idx[k] : tmp[s0 + k];
    const uint32_t dst = s0 + (canon ? rank_in(s_idx, n, src) : (uint32_t)k);
    if (src >= (uint32_t)p.nw) {
      set_status(S, RTS_E_DEVICE, -1);
      continue;
    }
    WP[dst] = make_float4(pos[src], pos[nw + src], pos[2 * nw + src], 0.0f);
    WID[dst] = src;
  }
}

// Byte fill of a device range (a kernel rather than hipMemsetAsync, so that
// set-up and resets stay plain kernel launches on the caller's stream).
__global__ void k_fill_bytes(uint8_t *p, uint8_t v, size_t bytes) {
  const uint32_t w = (uint32_t)v * 0x01010101u;
  const size_t words = bytes >> 2;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride)
    reinterpret_cast<uint32_t *>(p)[i] = w;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < (bytes & 3u)) p[(words << 2) + t] = v;
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
                     d.P[cur], d.ID[cur], d.KEYOLD, d.RANK, d.COUNT, d.CTRL, d.ACTN, d.S);
}
void launch_prep_scan(DevCtrl *ctrl, hipStream_t st) {
  hipLaunchKernelGGL(k_prep_scan, dim3(1), dim3(1), 0, st, ctrl);
}
void launch_scan(const DevParams &p, const DevPtrs &d, uint32_t *start, bool fluid,
                 hipStream_t st) {
  hipLaunchKernelGGL(k_scan, dim3(blocks_for(p.nb, kScanTile)), dim3(256), 0, st, d.COUNT, start,
                     p.nb, d.TILES, d.TILES2, fluid ? d.OCC : nullptr, d.OCCR, d.LRAW, d.LVL,
                     d.CTRL, d.S);
}
void launch_scatter(const DevParams &p, const DevPtrs &d, hipStream_t st) {
  if (p.n == 0) return;
  hipLaunchKernelGGL(k_scatter, dim3(blocks_for(p.n, 256)), dim3(256), 0, st, p.n, d.KEYOLD,
                     d.RANK, d.CELL_START, d.TMP, d.S);
}
void launch_cell_gather(const DevParams &p, const DevPtrs &d, int cur, int grid, hipStream_t st) {
  const int nx = cur ^ 1;
  hipLaunchKernelGGL(k_cell_gather, dim3((unsigned)grid), dim3(256), 0, st, p, d.OCCR, d.TMP, d.PERM, d.KEY, d.P[cur], d.V[cur], d.A[cur], d.M[cur],
                     d.ID[cur], d.P[nx], d.V[nx], d.A[nx], d.M[nx], d.ID[nx], d.LRAW, d.S);
}
void launch_rmin_flags(const DevParams &p, const DevPtrs &d, int cur, int do_flags, int grid,
                       hipStream_t st, const uint8_t *src) {
  hipLaunchKernelGGL(k_rmin_flags, dim3((unsigned)grid), dim3(256), 0, st, p, d.OCCR,
                     src ? src : d.LRAW, d.LVL, d.M[cur], d.P[cur], d.BLKU, d.BLKERR, d.BLKAMAX, d.ACT,
                     d.ACTN, d.S, do_flags);
}
void launch_search_density(const DevParams &p, const DevPtrs &d, int cur, int grid, int threads,
                           hipStream_t st) {
  auto go = [&](auto kernel, int nt) {
    hipLaunchKernelGGL(kernel, dim3((unsigned)grid), dim3((unsigned)nt), 0, st, p, d.ACT,
                       d.CELL_START, d.WCELL_START, d.P[cur], d.V[cur], d.M[cur], d.PRES, d.NNB,
                       d.LIST, d.WP, d.BLKU, d.BLKERR, d.ID[cur], d.ACTN, d.CTRL, d.S);
  };
  if (threads == 256) go(k_search_density<256>, 256);
  else go(k_search_density<512>, 512);
}
void launch_force(const DevParams &p, const DevPtrs &d, int cur, int grid, int lanes,
                  hipStream_t st) {
  auto go = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, dim3((unsigned)grid), dim3(kForceThreads), 0, st, p, d.ACT,
                       d.CELL_START, d.WCELL_START, d.P[cur], d.V[cur], d.M[cur], d.NNB, d.LIST,
                       d.WP, d.ANEW, d.BLKAMAX, d.ACTN, d.CTRL);
  };
  if (lanes == 4) go(k_force<4>);
  else go(k_force<8>);
}
void launch_step_stats(const DevParams &p, const DevPtrs &d, hipStream_t st) {
  hipLaunchKernelGGL(k_step_stats, dim3(kStatBlocks), dim3(256), 0, st, p, d.OCC, d.BLKU,
                     d.BLKERR, d.BLKAMAX, d.LVL, d.PART, d.CTRL, d.S);
}
void launch_stats_correct_predict(const DevParams &p, const DevPtrs &d, int cur,
                                  hipStream_t st) {
  const unsigned nb = blocks_for(p.n, 256);
  const unsigned grid = nb > (unsigned)kStatBlocks ? nb : (unsigned)kStatBlocks;
  hipLaunchKernelGGL(k_stats_correct_predict, dim3(grid), dim3(256), 0, st, p, d.OCC, d.BLKU,
                     d.BLKERR, d.BLKAMAX, d.LVL, d.PART, d.CTRL, d.S, d.P[cur], d.V[cur],
                     d.A[cur], d.M[cur], d.ANEW, d.ID[cur], d.KEYOLD, d.RANK, d.COUNT, d.ACTN);
}
void launch_correct_predict(const DevParams &p, const DevPtrs &d, int cur, hipStream_t st) {
  if (p.n == 0) return;
  hipLaunchKernelGGL(k_correct_predict, dim3(blocks_for(p.n, 256)), dim3(256), 0, st, p, d.P[cur],
                     d.V[cur], d.A[cur], d.M[cur], d.ANEW, d.S);
}
void launch_debug_lists(const DevParams &p, const DevPtrs &d, int cur, uint32_t *out,
                        uint32_t *out_n, hipStream_t st) {
  if (p.n == 0) return;
  hipLaunchKernelGGL(k_debug_lists, dim3(blocks_for(p.n, 256)), dim3(256), 0, st, p, d.KEY,
                     d.CELL_START, d.WCELL_START, d.M[cur], d.NNB, d.LIST, out, out_n);
}
void launch_set_state(const DevParams &p, const DevPtrs &d, int cur, const float *pos,
                      const float *vel, hipStream_t st) {
  if (p.n == 0) return;
  hipLaunchKernelGGL(k_set_state, dim3(blocks_for(p.n, 256)), dim3(256), 0, st, p, pos, vel,
                     d.P[cur], d.V[cur], d.A[cur], d.M[cur], d.ID[cur], d.PRES);
}
void launch_add_velocity(const DevParams &p, const DevPtrs &d, int cur, const float *dv,
                         hipStream_t st) {
  if (p.n == 0) return;
  hipLaunchKernelGGL(k_add_velocity, dim3(blocks_for(p.n, 256)), dim3(256), 0, st, p, dv,
                     d.ID[cur], d.V[cur]);
}
void launch_get_state(const DevParams &p, const DevPtrs &d, int cur, float *pos, float *vel,
                      float *acc, float *rho, float *pres, uint8_t *level, hipStream_t st) {
  launch_get_range(p, d, cur, 0u, (uint32_t)p.n, pos, vel, acc, rho, pres, level, st);
}
void launch_get_range(const DevParams &p, const DevPtrs &d, int cur, uint32_t lo, uint32_t cnt,
                      float *pos, float *vel, float *acc, float *rho, float *pres,
                      uint8_t *level, hipStream_t st) {
  if (p.n == 0 || cnt == 0) return;
  hipLaunchKernelGGL(k_get_state, dim3(blocks_for(p.n, 256)), dim3(256), 0, st, p, d.P[cur],
                     d.V[cur], d.A[cur], d.M[cur], d.ID[cur], lo, cnt, pos, vel, acc, rho, pres,
                     level);
}
void launch_init_lattice(const DevParams &p, const DevPtrs &d, uint32_t first, uint32_t cnt,
                         const LatticeSpec &L, hipStream_t st) {
  if (cnt == 0) return;
  hipLaunchKernelGGL(k_init_lattice, dim3(blocks_for((int)cnt, 256)), dim3(256), 0, st, p,
                     first, cnt, L, d.P[0], d.V[0], d.A[0], d.M[0], d.ID[0], d.PRES);
}
void launch_scene_stats(const DevParams &p, const DevPtrs &d, int cur, hipStream_t st) {
  launch_fill(d.SCN_STAT, 0, sizeof(SceneStat) * (size_t)p.n_scenes, st);
  if (p.n == 0) return;
  hipLaunchKernelGGL(k_scene_stats, dim3(blocks_for(p.n, 256)), dim3(256), 0, st, p, d.P[cur],
                     d.M[cur], d.ID[cur], d.NNB, d.SCN_OFF, d.SCN_STAT);
}
void launch_wall_sort(const DevParams &p, const DevPtrs &d, const float *pos, hipStream_t st) {
  launch_prep_scan(d.CTRL, st);
  if (p.nw > 0)
    hipLaunchKernelGGL(k_wall_keys, dim3(blocks_for(p.nw, 256)), dim3(256), 0, st, p, pos, d.WKEY,
                       d.WRANK, d.COUNT);
  launch_scan(p, d, d.WCELL_START, false, st);
  if (p.nw > 0) {
    hipLaunchKernelGGL(k_scatter, dim3(blocks_for(p.nw, 256)), dim3(256), 0, st, p.nw, d.WKEY,
                       d.WRANK, d.WCELL_START, d.WTMP, d.S);
    hipLaunchKernelGGL(k_wall_gather, dim3((unsigned)p.nb), dim3(64), 0, st, p, d.WCELL_START,
                       d.WTMP, pos, d.WP, d.WID, d.S);
  }
}
void launch_fill(void *p, uint8_t v, size_t bytes, hipStream_t st) {
  if (bytes == 0) return;
  const size_t words = (bytes + 3) / 4;
  const unsigned grid = (unsigned)(words < 256 * 1024 ? (words + 255) / 256 : 1024);
  hipLaunchKernelGGL(k_fill_bytes, dim3(grid), dim3(256), 0, st, (uint8_t *)p, v, bytes);
}
void launch_reset_scalars(DevScalars *S, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_scalars, dim3(1), dim3(1), 0, st, S);
}

}  // namespace rts
