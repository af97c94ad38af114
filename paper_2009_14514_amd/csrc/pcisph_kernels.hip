// HIP kernels of PCISPH with regional iteration counts on gfx950 (Goswami &
// Batty, Section 5, Algorithms 2 and 3).
//
// A major step sorts the particles into a grid of edge 1.1 r once (the sort
// kernels of the WCSPH path), assigns regions R_1..R_4 (block levels 0..3)
// from Eq. 2-3, grows regions 1 and 2 by a few block layers, smooths with
// R_min and marks the observed blocks.  Each minor step then
//   lists        rebuilds the neighbour lists of particles whose validity ran
//                out, against the grid of the major step (two block layers
//                for region 1, or regions 1 and 2)
//   nonpressure  sums their gravity + viscosity over the new lists
//   reset        p = 0, F^p = 0, S_e empty
//   per iteration (the host reads the error reductions between iterations):
//     predict    v* = v + dt (a_vg + a_p), x* = x + dt v*   (all)
//     density    rho*, error, p += delta (rho* - rho0)      (turn, S_e, observed)
//     mark_se    blocks around S_e particles join the observed set
//     force      pressure acceleration                      (turn, S_e)
//     errstats   max and mean compression, region counts
//   integrate    symplectic Euler, validity, requests for smaller steps
//   demote       blocks (and their particles) take the requested steps
//
// Density and pressure force run one thread per particle: the lists hold
// about 45 entries within 1.1 r and neighbouring threads share most of them,
// so gathers hit the caches (each XCD takes one contiguous range of
// particles, so neighbours share its L2).  The list pass sweeps a wave's
// eight particles' rows together, a candidate per lane.  Sums run in list
// order and the reductions are folded in a fixed order: runs are
// deterministic.
#include "rts_device.h"
#include "xcd.h"

namespace rts {

constexpr uint32_t kNoLevel = 0xFFFFFFFFu;

// Neighbour lists in quads: entries 4q .. 4q+3 of particle i are the four
// words at (q n + i) 4, so a lane reads four entries with one 16-byte load
// and the 64 lanes of a wave read consecutive quads (the passes over the
// lists are bound by issuing loads, not by bytes).
__device__ inline size_t list_word(uint32_t i, uint32_t k, size_t ncap) {
  return ((size_t)(k >> 2) * ncap + i) * 4u + (k & 3u);
}

__device__ inline int region_validity(int level, int major_len) {
  // neighbourhoods: region 1 every minor step, region 2 every second one,
  // regions 3 and 4 at the next major step
  return level <= 1 ? level + 1 : major_len;
}

__device__ inline bool has_turn(uint32_t turn, uint32_t level) { return (turn >> level) & 1u; }

// ---------------------------------------------------------------------------
// major step: region dilation, observed blocks, particle flags
// ---------------------------------------------------------------------------
// Dilation of `level` by a cube of `layers` blocks, separated into x, y, z
// passes over occupancy masks (exact for the Chebyshev cube).
__global__ void k_pci_dil_x(DevParams p, const uint8_t *__restrict__ src, uint8_t *__restrict__ m1,
                            int level, int layers) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= p.nb) return;
  const int3 c = coords_of(p, (uint32_t)b);
  uint8_t hit = 0;
  for (int dx = -layers; dx <= layers; ++dx) {
    const int x = c.x + dx;
    if (x >= 0 && x < p.nc[0] && src[b + dx] == (uint8_t)level) hit = 1;
  }
  m1[b] = hit;
}
__global__ void k_pci_dil_y(DevParams p, const uint8_t *__restrict__ m1, uint8_t *__restrict__ m2,
                            int layers) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= p.nb) return;
  const int3 c = coords_of(p, (uint32_t)b);
  uint8_t hit = 0;
  for (int dy = -layers; dy <= layers; ++dy) {
    const int y = c.y + dy;
    if (y >= 0 && y < p.nc[1] && m1[b + dy * p.nc[0]]) hit = 1;
  }
  m2[b] = hit;
}
__global__ void k_pci_dil_z(DevParams p, const uint8_t *__restrict__ m2,
                            const uint8_t *__restrict__ src, uint8_t *__restrict__ dst, int level,
                            int layers) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= p.nb) return;
  const int3 c = coords_of(p, (uint32_t)b);
  const int plane = p.nc[0] * p.nc[1];
  uint8_t hit = 0;
  for (int dz = -layers; dz <= layers; ++dz) {
    const int z = c.z + dz;
    if (z >= 0 && z < p.nc[2] && m2[b + dz * plane]) hit = 1;
  }
  const uint8_t l = src[b];
  dst[b] = (l != kEmpty && l > (uint8_t)level && hit) ? (uint8_t)level : l;
}

// Observed blocks (Section 5, local density correction): occupied blocks
// with an occupied neighbour of a smaller region.
__global__ void k_pci_observed(DevParams p, const uint32_t *__restrict__ occ,
                               const uint8_t *__restrict__ lvl, uint8_t *__restrict__ ob,
                               const DevScalars *__restrict__ S) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= S->n_occ) return;
  const uint32_t b = occ[q];
  const int3 c = coords_of(p, b);
  const uint8_t own = lvl[b];
  uint8_t o = 0;
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int x = c.x + dx, y = c.y + dy, z = c.z + dz;
        if (x < 0 || y < 0 || z < 0 || x >= p.nc[0] || y >= p.nc[1] || z >= p.nc[2]) continue;
        if (lvl[(uint32_t)(x + p.nc[0] * (y + p.nc[1] * z))] < own) o = 1;
      }
  ob[b] = o;
}

// Algorithm 2: every particle takes its block's region and rebuilds its
// neighbourhood at the start of a major step.
__global__ void k_pci_major_flags(DevParams p, const uint32_t *__restrict__ key,
                                  const uint8_t *__restrict__ lvl, uint32_t *__restrict__ M,
                                  int major_len) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  const uint32_t l = lvl[key[i]];
  M[i] = meta_pack(l, 1u, 0u, region_validity((int)l, major_len));
}

// ---------------------------------------------------------------------------
// minor step
// ---------------------------------------------------------------------------
// dW/dr / r, so that grad W(x_ij) = f * x_ij
__device__ inline float grad_factor(const DevParams &p, float r2) {
  const float r = __builtin_sqrtf(r2);
  return p.sigma * p.inv_h * dw_shape(r * p.inv_h) / r;
}

// Neighbour lists against the grid of the major step (Section 5,
// neighbourhood computation): blocks up to `rings` layers around the
// particle's block, float predicate with the list radius, canonical order
// (fluid by sorted index, then walls by wall sorted index | bit 31).
//
// A wave takes kPciWave consecutive particles of the sorted order.  When the
// ones that rebuild their lists search one block layer and share a block row
// (y, z) within two neighbouring blocks in x (most waves: a block holds about
// 11 particles), the wave sweeps the union of their rows once, a candidate per
// lane, and tests every particle against each chunk of 64: each candidate is
// loaded once per wave instead of once per particle.  A candidate counts for
// a particle only inside the particle's own 27 blocks (its block in x from
// the row's block starts), so each list holds exactly its own rows' hits, in
// candidate order.  Other waves give each particle kPciSub lanes, which load
// kPciSub consecutive candidates of a row at once; a ballot of their hits
// places each hit, so the list keeps the canonical order either way.
constexpr int kPciSub = 8;
constexpr int kPciWave = 64 / kPciSub;   // particles per wave, both ways

// One particle's list with kPciSub lanes (lane sub of the group starting at
// lane `first`).
__device__ inline void pci_list_lanes(const DevParams &p, const float4 *__restrict__ P,
                                      const uint32_t *__restrict__ key,
                                      const uint32_t *__restrict__ start,
                                      const float4 *__restrict__ WP,
                                      const uint32_t *__restrict__ wstart,
                                      uint32_t *__restrict__ nbr, uint32_t *__restrict__ nnb,
                                      const uint32_t *__restrict__ ids, DevScalars *S, uint32_t i,
                                      int rings, uint32_t sub, uint32_t first) {
  const float4 xi = P[i];
  const int3 c = coords_of(p, key[i]);
  const size_t ncap = (size_t)p.ncap;
  uint32_t cnt = 0;  // the same in the particle's lanes
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1 && p.nw == 0) break;
    const uint32_t *cs = pass == 0 ? start : wstart;
    const float4 *X = pass == 0 ? P : WP;
    const uint32_t tag = pass == 0 ? 0u : kWallBit;
    for (int dz = -rings; dz <= rings; ++dz) {
      const int z = c.z + dz;
      if (z < 0 || z >= p.nc[2]) continue;
      for (int dy = -rings; dy <= rings; ++dy) {
        const int y = c.y + dy;
        if (y < 0 || y >= p.nc[1]) continue;
        const int x0 = max(c.x - rings, 0), x1 = min(c.x + rings, p.nc[0] - 1);
        const uint32_t row = (uint32_t)p.nc[0] * ((uint32_t)y + (uint32_t)p.nc[1] * (uint32_t)z);
        const uint32_t s0 = cs[row + (uint32_t)x0], s1 = cs[row + (uint32_t)x1 + 1u];
        for (uint32_t base = s0; base < s1; base += kPciSub) {
          const uint32_t j = base + sub;
          bool hit = false;
          if (j < s1 && !(pass == 0 && j == i)) {
            const float4 q = X[j];
            hit = dist2_exact(xi.x, xi.y, xi.z, q.x, q.y, q.z) < p.r2l;
          }
          // the group's hits among these candidates, in candidate order
          const uint32_t mask = (uint32_t)(__ballot(hit) >> first) & ((1u << kPciSub) - 1u);
          if (hit) {
            const uint32_t pos = cnt + (uint32_t)__popc(mask & ((1u << sub) - 1u));
            if (pos < (uint32_t)p.nbr_cap) nbr[list_word(i, pos, ncap)] = j | tag;
          }
          cnt += (uint32_t)__popc(mask);
        }
      }
    }
  }
  if (sub != 0) return;
  if (cnt > (uint32_t)p.nbr_cap) {
    set_status(S, RTS_E_CAPACITY, (int32_t)ids[i]);
    cnt = (uint32_t)p.nbr_cap;
  }
  nnb[i] = cnt;
}

// The union rows of a wave's particles, one pass (fluid or walls): row r
// (dz = r / 3 - 1, dy = r % 3 - 1) holds the candidates from rs[r] on, at
// positions off[r] .. off[r + 1] of the sweep; b[r] are the first sorted
// indices of its second, third and fourth block in x (or its end).
struct PciRows {
  uint4 rb[9];        // rs, b1, b2, b3
  uint32_t off[10];
};
// List entries a wave's particle gathers in LDS before they are stored in
// quads: the shared sweep runs when the list capacity fits.
constexpr int kPciLdsCap = 128;

__global__ void __launch_bounds__(256) k_pci_lists(
    DevParams p, const float4 *__restrict__ P, const uint32_t *__restrict__ M,
    const uint32_t *__restrict__ key, const uint32_t *__restrict__ start,
    const float4 *__restrict__ WP, const uint32_t *__restrict__ wstart,
    uint32_t *__restrict__ nbr, uint32_t *__restrict__ nnb, const uint32_t *__restrict__ ids,
    DevScalars *S) {
  __shared__ PciRows s_rows[4];
  __shared__ uint32_t s_list[4][kPciWave][kPciLdsCap];
  __shared__ float4 s_mem[4][kPciWave];   // the wave's particles: x, y, z, block x
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  const uint32_t i0 = (xcd_block(blockIdx.x, gridDim.x) * 4u + wave) * (uint32_t)kPciWave;
  if (i0 >= (uint32_t)p.n) return;
  // the wave's particles, one per lane below kPciWave
  const uint32_t im = i0 + (lane & (uint32_t)(kPciWave - 1));
  bool mem = false;
  int rings = 1;
  int3 c = make_int3(0, 0, 0);
  float4 xm = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if (lane < (uint32_t)kPciWave && im < (uint32_t)p.n) {
    const uint32_t m = M[im];
    if (meta_compute(m)) {
      mem = true;
      rings = (p.mode == RTS_MODE_RTS && (int)meta_level(m) < p.two_ring_levels) ? 2 : 1;
      c = coords_of(p, key[im]);
      xm = P[im];
    }
  }
  const uint32_t memmask = (uint32_t)__ballot(mem);
  if (memmask == 0u) return;
  const int lead = __ffs((int)memmask) - 1;
  const int cy = __shfl(c.y, lead, 64), cz = __shfl(c.z, lead, 64);
  int xmn = mem ? c.x : 0x7FFFFFFF, xmx = mem ? c.x : -1;
#pragma unroll
  for (int o = 1; o < kPciWave; o <<= 1) {
    xmn = min(xmn, __shfl_xor(xmn, o, 64));
    xmx = max(xmx, __shfl_xor(xmx, o, 64));
  }
  xmn = __builtin_amdgcn_readfirstlane(xmn);
  xmx = __builtin_amdgcn_readfirstlane(xmx);
  const bool odd = mem && (rings != 1 || c.y != cy || c.z != cz);
  if (__ballot(odd) != 0ull || xmx - xmn > 1 || p.nbr_cap > kPciLdsCap) {
    // the particle's own kPciSub lanes; a particle's lanes leave together
    const uint32_t i = i0 + lane / (uint32_t)kPciSub;
    if (i >= (uint32_t)p.n) return;
    const uint32_t m = M[i];
    if (!meta_compute(m)) return;
    const int ri = (p.mode == RTS_MODE_RTS && (int)meta_level(m) < p.two_ring_levels) ? 2 : 1;
    pci_list_lanes(p, P, key, start, WP, wstart, nbr, nnb, ids, S, i, ri,
                   lane & (uint32_t)(kPciSub - 1), lane & ~(uint32_t)(kPciSub - 1));
    return;
  }
  // one sweep of the union rows for every particle of the wave
  const size_t ncap = (size_t)p.ncap;
  const int xlo = max(xmn - 1, 0), xhi = min(xmx + 1, p.nc[0] - 1);
  if (lane < (uint32_t)kPciWave)
    s_mem[wave][lane] = make_float4(xm.x, xm.y, xm.z, __builtin_bit_cast(float, c.x));
  uint32_t cnt[kPciWave];
#pragma unroll
  for (int t = 0; t < kPciWave; ++t) cnt[t] = 0u;
  PciRows &rows = s_rows[wave];
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1 && p.nw == 0) break;
    const uint32_t *cs = pass == 0 ? start : wstart;
    const float4 *X = pass == 0 ? P : WP;
    const uint32_t tag = pass == 0 ? 0u : kWallBit;
    // row r in lane r: its range and the block starts inside it
    uint32_t len = 0;
    uint4 rb = make_uint4(0u, 0u, 0u, 0u);
    if (lane < 9u) {
      const int y = cy + (int)(lane % 3u) - 1, z = cz + (int)(lane / 3u) - 1;
      if (y >= 0 && y < p.nc[1] && z >= 0 && z < p.nc[2]) {
        const uint32_t row = (uint32_t)p.nc[0] * ((uint32_t)y + (uint32_t)p.nc[1] * (uint32_t)z);
        const uint32_t s0 = cs[row + (uint32_t)xlo], s1 = cs[row + (uint32_t)xhi + 1u];
        const uint32_t e1 = xlo + 1 <= xhi ? cs[row + (uint32_t)xlo + 1u] : s1;
        const uint32_t e2 = xlo + 2 <= xhi ? cs[row + (uint32_t)xlo + 2u] : s1;
        const uint32_t e3 = xlo + 3 <= xhi ? cs[row + (uint32_t)xlo + 3u] : s1;
        rb = make_uint4(s0, e1, e2, e3);
        len = s1 - s0;
      }
    }
    uint32_t incl = len;
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
      const uint32_t u = (uint32_t)__shfl_up((int)incl, o, 64);
      if (lane >= (uint32_t)o) incl += u;
    }
    if (lane < 9u) {
      rows.rb[lane] = rb;
      rows.off[lane] = incl - len;
    }
    if (lane == 8u) rows.off[9] = incl;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    uint32_t off[10];
#pragma unroll
    for (int r = 0; r < 10; ++r) off[r] = __builtin_amdgcn_readfirstlane(rows.off[r]);
    const uint32_t total = off[9];
    // candidate at sweep position pos: its sorted index and its block in x
    // (far away and in no particle's blocks past the end)
    const auto candidate = [&](uint32_t pos, uint32_t &j, int &cbx) {
      uint32_t r = 0;
#pragma unroll
      for (int k = 1; k < 9; ++k) r += pos >= off[k] ? 1u : 0u;
      const uint4 rr = rows.rb[r];
      j = rr.x + (pos - rows.off[r]);
      cbx = xlo + (j >= rr.y ? 1 : 0) + (j >= rr.z ? 1 : 0) + (j >= rr.w ? 1 : 0);
      float4 q = make_float4(1e30f, 1e30f, 1e30f, 0.0f);
      if (pos < total) q = X[j];
      else cbx = -4;
      return q;
    };
    // the wave's particles in block xmn (bit t set), the others in xmx
    uint32_t in_mn = 0;
#pragma unroll
    for (int t = 0; t < kPciWave; ++t)
      in_mn |= (__builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, s_mem[wave][t].w)) == xmn
                    ? 1u
                    : 0u)
               << t;
    // two chunks in flight, each loaded into the registers it is tested from
    const auto test_chunk = [&](const float4 q, const uint32_t j, const int cbx) {
      // inside the 27 blocks of a particle in block xmn, or of one in xmx
      const bool okn = (uint32_t)(cbx - xmn + 1) <= 2u;
      const bool okx = (uint32_t)(cbx - xmx + 1) <= 2u;
#pragma unroll
      for (int t = 0; t < kPciWave; ++t) {
        // every slot is tested (no branch); a slot that is not one of the
        // wave's particles never hits
        const uint32_t it = i0 + (uint32_t)t;
        const float4 mt = s_mem[wave][t];
        const bool ok = ((in_mn >> t) & 1u) ? okn : okx;
        const bool hit = (((memmask >> t) & 1u) != 0u) & ok & !(pass == 0 && j == it) &
                         (dist2_exact(mt.x, mt.y, mt.z, q.x, q.y, q.z) < p.r2l);
        const unsigned long long hm = __ballot(hit);
        if (hit) {
          const uint32_t at = __builtin_amdgcn_mbcnt_hi(
              (uint32_t)(hm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)hm, cnt[t]));
          if (at < (uint32_t)p.nbr_cap) s_list[wave][t][at] = j | tag;
        }
        cnt[t] += (uint32_t)__popcll(hm);
      }
    };
    uint32_t ja, jb;
    int ba, bb;
    float4 qa = candidate(lane, ja, ba);
    float4 qb = candidate(64u + lane, jb, bb);  // not tested when total <= 64
    for (uint32_t pos0 = 0; pos0 < total; pos0 += 128u) {
      test_chunk(qa, ja, ba);
      if (pos0 + 128u < total) qa = candidate(pos0 + 128u + lane, ja, ba);
      if (pos0 + 64u >= total) break;
      test_chunk(qb, jb, bb);
      if (pos0 + 192u < total) qb = candidate(pos0 + 192u + lane, jb, bb);
    }
    // the next pass rewrites the rows
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  // the gathered entries, a quad per lane (entries past the list's end are
  // stored as 0)
  uint32_t nq[kPciWave], qoff[kPciWave + 1];
  qoff[0] = 0u;
#pragma unroll
  for (int t = 0; t < kPciWave; ++t) {
    const uint32_t n = min(cnt[t], (uint32_t)p.nbr_cap);
    nq[t] = ((memmask >> t) & 1u) ? (n + 3u) / 4u : 0u;
    qoff[t + 1] = qoff[t] + nq[t];
  }
  for (uint32_t k0 = 0; k0 < qoff[kPciWave]; k0 += 64u) {
    const uint32_t k = k0 + lane;
    if (k >= qoff[kPciWave]) break;
    uint32_t t = 0;
#pragma unroll
    for (int u = 1; u < kPciWave; ++u) t += k >= qoff[u] ? 1u : 0u;
    uint32_t q = k, n = 0;
#pragma unroll
    for (int u = 0; u < kPciWave; ++u)
      if (t == (uint32_t)u) {
        q = k - qoff[u];
        n = min(cnt[u], (uint32_t)p.nbr_cap);
      }
    const uint32_t e = 4u * q;
    const uint32_t *row = s_list[wave][t];
    const uint4 v = make_uint4(row[e], e + 1u < n ? row[e + 1u] : 0u, e + 2u < n ? row[e + 2u] : 0u,
                               e + 3u < n ? row[e + 3u] : 0u);
    *reinterpret_cast<uint4 *>(nbr + list_word(i0 + t, e, ncap)) = v;
  }
  // lane t writes particle t's count
  uint32_t mine = 0;
#pragma unroll
  for (int t = 0; t < kPciWave; ++t)
    if (lane == (uint32_t)t) mine = cnt[t];
  if (!mem) return;
  if (mine > (uint32_t)p.nbr_cap) {
    set_status(S, RTS_E_CAPACITY, (int32_t)ids[im]);
    mine = (uint32_t)p.nbr_cap;
  }
  nnb[im] = mine;
}

// Non-pressure acceleration of Algorithm 2 for the particles that rebuilt
// their lists: gravity plus the artificial viscosity of approaching pairs
// within the support, summed over the list in list order (walls at rest).
__global__ void __launch_bounds__(256) k_pci_nonpressure(
    DevParams p, const float4 *__restrict__ P, const float4 *__restrict__ V,
    const uint32_t *__restrict__ M, const uint32_t *__restrict__ nbr,
    const uint32_t *__restrict__ nnb, const float4 *__restrict__ WP, float4 *__restrict__ fvg) {
  const int i = (int)(xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x);
  if (i >= p.n) return;
  if (!meta_compute(M[i])) return;
  const float4 xi = P[i], vi = V[i];
  const float rs2 = p.support * p.support;
  const uint4 *L4 = reinterpret_cast<const uint4 *>(nbr) + i;
  const size_t stride = (size_t)p.ncap;
  const uint32_t n = nnb[i];
  float ax = 0.0f, ay = 0.0f, az = 0.0f;
  auto add = [&](const float4 q, const float4 u) {
    const float dx = xi.x - q.x, dy = xi.y - q.y, dz = xi.z - q.z;
    const float r2 = dx * dx + dy * dy + dz * dz;
    const float vx = (vi.x - u.x) * dx + (vi.y - u.y) * dy + (vi.z - u.z) * dz;
    if (r2 > 0.0f && r2 < rs2 && vx < 0.0f) {
      const float pij = -p.pci_nu * vx * __builtin_amdgcn_rcpf(r2 + p.visc_eps_h2);
      const float sc = -p.mass * pij * grad_factor(p, r2);
      ax += sc * dx;
      ay += sc * dy;
      az += sc * dz;
    }
  };
  const uint32_t nfull = n & ~3u;
  for (uint32_t k0 = 0; k0 < nfull; k0 += 4) {
    // a full quad: its gathers are issued before they are used
    const uint4 e = L4[(size_t)(k0 >> 2) * stride];
    const uint32_t js[4] = {e.x, e.y, e.z, e.w};
    float4 q[4], u[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const bool wall = (js[k] & kWallBit) != 0u;
      q[k] = wall ? WP[js[k] & ~kWallBit] : P[js[k]];
      u[k] = wall ? make_float4(0.0f, 0.0f, 0.0f, 0.0f) : V[js[k]];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) add(q[k], u[k]);
  }
  if (nfull < n) {
    const uint4 e = L4[(size_t)(nfull >> 2) * stride];
    const uint32_t js[3] = {e.x, e.y, e.z};
    for (uint32_t k = 0; nfull + k < n; ++k) {
      const bool wall = (js[k] & kWallBit) != 0u;
      add(wall ? WP[js[k] & ~kWallBit] : P[js[k]],
          wall ? make_float4(0.0f, 0.0f, 0.0f, 0.0f) : V[js[k]]);
    }
  }
  fvg[i] = make_float4(p.g[0] + ax, p.g[1] + ay, p.g[2] + az, 0.0f);
}

__global__ void k_pci_reset(DevParams p, float4 *__restrict__ pv, float4 *__restrict__ fp,
                            float *__restrict__ pq, uint8_t *__restrict__ se,
                            uint8_t *__restrict__ nearse) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < p.n) {
    pv[i] = make_float4(0.0f, 0.0f, 0.0f, p.rho0);
    fp[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    pq[i] = 0.0f;
    se[i] = 0;
  }
  if (i < p.nb) nearse[i] = 0;
}

__global__ void k_pci_predict(DevParams p, const float4 *__restrict__ P,
                              const float4 *__restrict__ V, const float4 *__restrict__ fvg,
                              const float4 *__restrict__ fp, const float *__restrict__ pq,
                              float4 *__restrict__ xs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  const float4 x = P[i], v = V[i], a = fvg[i], b = fp[i];
  const float dt = p.dt_base;
  const float vx = v.x + dt * (a.x + b.x), vy = v.y + dt * (a.y + b.y), vz = v.z + dt * (a.z + b.z);
  // w carries p / rho*^2, so the pressure-force pass gathers one float4 per
  // neighbour; the density pass updates it for the particles it evaluates
  xs[i] = make_float4(x.x + dt * vx, x.y + dt * vy, x.z + dt * vz, pq[i]);
}

// Algorithm 3, density prediction: particles with the turn, S_e and the
// observed blocks.  rho* = m (W(0) + sum_j W + sum_walls W); the relative
// excess is formed as (m sigma / rho0) ((sum - c_hi) - (comp + c_lo)) with
// c = rho0 / (m sigma) - 1, before any rounding to rho*.
__global__ void __launch_bounds__(256) k_pci_density(
    DevParams p, float4 *__restrict__ xs, float4 *__restrict__ pv, float *__restrict__ pq,
    const uint32_t *__restrict__ M, const uint32_t *__restrict__ key,
    const uint8_t *__restrict__ ob, const uint8_t *__restrict__ nearse,
    uint8_t *__restrict__ se, const uint32_t *__restrict__ nbr, const uint32_t *__restrict__ nnb,
    const float4 *__restrict__ WP, uint32_t turn) {
  const int i = (int)(xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x);
  if (i >= p.n) return;
  const uint32_t b = key[i];
  const bool in_se = se[i] != 0;
  if (!(has_turn(turn, meta_level(M[i])) || in_se || ob[b] || nearse[b])) return;
  const float4 xi = xs[i];
  const uint4 *L4 = reinterpret_cast<const uint4 *>(nbr) + i;
  const size_t stride = (size_t)p.ncap;
  const uint32_t n = nnb[i];
  float sum = 0.0f, comp = 0.0f;
  auto add = [&](const float4 q) {
    const float dx = xi.x - q.x, dy = xi.y - q.y, dz = xi.z - q.z;
    const float r2 = dx * dx + dy * dy + dz * dz;
    const float w = w_shape(__builtin_sqrtf(r2) * p.inv_h);
    const float y = w - comp;
    const float t = sum + y;
    comp = (t - sum) - y;
    sum = t;
  };
  // a neighbour's position: a wall's from the wall array (one load either way)
  auto pos = [&](uint32_t j) {
    return *((j & kWallBit) ? WP + (j & ~kWallBit) : xs + j);
  };
  const uint32_t nfull = n & ~3u;
  for (uint32_t k0 = 0; k0 < nfull; k0 += 4) {
    // a full quad: its four gathers are issued before they are used
    const uint4 e = L4[(size_t)(k0 >> 2) * stride];
    const float4 q0 = pos(e.x), q1 = pos(e.y), q2 = pos(e.z), q3 = pos(e.w);
    add(q0);
    add(q1);
    add(q2);
    add(q3);
  }
  if (nfull < n) {
    const uint4 e = L4[(size_t)(nfull >> 2) * stride];
    const uint32_t js[3] = {e.x, e.y, e.z};
    for (uint32_t u = 0; nfull + u < n; ++u) add(pos(js[u]));
  }
  const float dev = p.kms * ((sum - p.c_hi) - (comp + p.c_lo));
  const float rho = p.rho0 + p.rho0 * dev;
  float4 s = pv[i];
  const float pn = s.x + p.delta * (p.rho0 * dev);
  s.x = pn > 0.0f ? pn : 0.0f;
  s.y = dev;
  s.w = rho;
  pv[i] = s;
  const float q = s.x / (rho * rho);
  pq[i] = q;
  // only the w word: other threads read this particle's x* meanwhile
  reinterpret_cast<float *>(xs + i)[3] = q;
  if (dev > p.eta_half) se[i] = 1;
}

// S_ob gains the blocks holding or bordering an S_e particle.
__global__ void k_pci_mark_se(DevParams p, const uint8_t *__restrict__ se,
                              const uint32_t *__restrict__ key, uint8_t *__restrict__ nearse) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n || !se[i]) return;
  const int3 c = coords_of(p, key[i]);
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int x = c.x + dx, y = c.y + dy, z = c.z + dz;
        if (x < 0 || y < 0 || z < 0 || x >= p.nc[0] || y >= p.nc[1] || z >= p.nc[2]) continue;
        nearse[(uint32_t)(x + p.nc[0] * (y + p.nc[1] * z))] = 1;
      }
}

// Pressure acceleration -m sum_j (p_i/rho_i^2 + p_j/rho_j^2) grad W(x*_ij);
// a wall particle mirrors p_i and rho_i.
__global__ void __launch_bounds__(256) k_pci_force(
    DevParams p, const float4 *__restrict__ xs,
    const uint32_t *__restrict__ M, const uint8_t *__restrict__ se,
    const uint32_t *__restrict__ nbr, const uint32_t *__restrict__ nnb,
    const float4 *__restrict__ WP, float4 *__restrict__ fp, uint32_t turn) {
  const int i = (int)(xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x);
  if (i >= p.n) return;
  if (!(has_turn(turn, meta_level(M[i])) || se[i])) return;
  const float4 xi = xs[i];
  const float qi = xi.w;
  const uint4 *L4 = reinterpret_cast<const uint4 *>(nbr) + i;
  const size_t stride = (size_t)p.ncap;
  const uint32_t n = nnb[i];
  const float rs2 = p.support * p.support;
  float ax = 0.0f, ay = 0.0f, az = 0.0f;
  auto add = [&](uint32_t j, const float4 q) {
    const float dx = xi.x - q.x, dy = xi.y - q.y, dz = xi.z - q.z;
    const float r2 = dx * dx + dy * dy + dz * dz;
    if (!(r2 > 0.0f) || r2 >= rs2) return;
    const float s = -p.mass * (qi + ((j & kWallBit) ? qi : q.w)) * grad_factor(p, r2);
    ax += s * dx;
    ay += s * dy;
    az += s * dz;
  };
  // one load per neighbour: x* with p / rho*^2 in w (a wall mirrors p_i, rho_i)
  auto pos = [&](uint32_t j) {
    return *((j & kWallBit) ? WP + (j & ~kWallBit) : xs + j);
  };
  const uint32_t nfull = n & ~3u;
  for (uint32_t k0 = 0; k0 < nfull; k0 += 4) {
    const uint4 e = L4[(size_t)(k0 >> 2) * stride];
    const float4 q0 = pos(e.x), q1 = pos(e.y), q2 = pos(e.z), q3 = pos(e.w);
    add(e.x, q0);
    add(e.y, q1);
    add(e.z, q2);
    add(e.w, q3);
  }
  if (nfull < n) {
    const uint4 e = L4[(size_t)(nfull >> 2) * stride];
    const uint32_t js[3] = {e.x, e.y, e.z};
    for (uint32_t u = 0; nfull + u < n; ++u) add(js[u], pos(js[u]));
  }
  fp[i] = make_float4(ax, ay, az, 0.0f);
}

// Max and mean compression over all particles (each keeps its latest
// error) and particles per region; per-workgroup partials folded in a fixed
// order by the last workgroup.
__device__ inline void pci_part_add(PciPart &t, const PciPart &u) {
  t.errmax = fmaxf(t.errmax, u.errmax);
  t.v2max = fmaxf(t.v2max, u.v2max);
  t.a2max = fmaxf(t.a2max, u.a2max);
  t.sum += u.sum;
  t.ncomp += u.ncomp;
  for (int k = 0; k < 4; ++k) t.hist[k] += u.hist[k];
}

// Reduces a 256-thread workgroup's partials (one per thread) in a fixed
// order: waves by shuffles, then the four wave totals in order.
__device__ inline PciPart pci_block_reduce(PciPart t, PciPart *s_w) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) {
    t.errmax = fmaxf(t.errmax, __shfl_xor(t.errmax, o, 64));
    t.v2max = fmaxf(t.v2max, __shfl_xor(t.v2max, o, 64));
    t.a2max = fmaxf(t.a2max, __shfl_xor(t.a2max, o, 64));
    t.sum += __shfl_xor(t.sum, o, 64);
    t.ncomp += __shfl_xor(t.ncomp, o, 64);
#pragma unroll
    for (int k = 0; k < 4; ++k) t.hist[k] += __shfl_xor(t.hist[k], o, 64);
  }
  if (lane == 0) s_w[wave] = t;
  __syncthreads();
  PciPart a = s_w[0];
  for (int w = 1; w < 4; ++w) pci_part_add(a, s_w[w]);
  __syncthreads();
  return a;
}

// Max and mean compression over all particles (each keeps its latest
// error), particles per region and with the compute flag; per-workgroup
// partials folded in a fixed order by the last workgroup.  `first`: the
// compute count is also kept as this minor step's list count.  With V and A
// given, also the largest |v|^2 and |a|^2 (the adaptive base step's bounds).
__global__ void __launch_bounds__(256) k_pci_errstats(DevParams p, const float4 *__restrict__ pv,
                                                     const uint32_t *__restrict__ M,
                                                     const float4 *__restrict__ V,
                                                     const float4 *__restrict__ A,
                                                     PciPart *__restrict__ part, DevPci *pci,
                                                     int first) {
  __shared__ PciPart s_w[4];
  __shared__ uint32_t s_last;
  const int tid = threadIdx.x;
  PciPart t = {};
  const auto take = [&](float e, uint32_t m) {
    e = fmaxf(e, 0.0f);
    t.errmax = fmaxf(t.errmax, e);
    t.sum += (double)e;
    const uint32_t l = meta_level(m);
    t.ncomp += (int32_t)meta_compute(m);
#pragma unroll
    for (int k = 0; k < 4; ++k) t.hist[k] += l == (uint32_t)k ? 1 : 0;
  };
  const int stride = (int)(gridDim.x * blockDim.x);
  int i = (int)(blockIdx.x * blockDim.x) + tid;
  if (!V) {
    // four particles' loads issued before any is used
    for (; i + 3 * stride < p.n; i += 4 * stride) {
      const float e0 = pv[i].y, e1 = pv[i + stride].y, e2 = pv[i + 2 * stride].y,
                  e3 = pv[i + 3 * stride].y;
      const uint32_t m0 = M[i], m1 = M[i + stride], m2 = M[i + 2 * stride], m3 = M[i + 3 * stride];
      take(e0, m0);
      take(e1, m1);
      take(e2, m2);
      take(e3, m3);
    }
  }
  for (; i < p.n; i += stride) {
    if (V) {
      const float4 v = V[i], a = A[i];
      t.v2max = fmaxf(t.v2max, norm2_exact(v.x, v.y, v.z));
      t.a2max = fmaxf(t.a2max, norm2_exact(a.x, a.y, a.z));
    }
    take(pv[i].y, M[i]);
  }
  const PciPart a = pci_block_reduce(t, s_w);
  if (tid == 0) {
    part[blockIdx.x] = a;
    __threadfence();
    s_last = atomicAdd(&pci->ticket, 1u) == gridDim.x - 1 ? 1u : 0u;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  // the last workgroup folds the partials: thread k takes partials k, k+256, ...
  PciPart u = {};
  for (unsigned g = (unsigned)tid; g < gridDim.x; g += 256) pci_part_add(u, part[g]);
  const PciPart r = pci_block_reduce(u, s_w);
  if (tid != 0) return;
  pci->ncomp = r.ncomp;
  if (first) pci->ncomp_first = r.ncomp;
  pci->errmax = r.errmax;
  pci->avg = p.n > 0 ? r.sum / (double)p.n : 0.0;
  for (int k = 0; k < 4; ++k) pci->hist[k] = r.hist[k];
  if (V) {
    pci->v2max = r.v2max;
    pci->a2max = r.a2max;
  }
  pci->ticket = 0u;
}

// Pressure snapshot before local iterations, or its restoration.
__global__ void k_pci_pressure_copy(DevParams p, float4 *__restrict__ pv, float *__restrict__ pq,
                                    int to_backup) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  float4 s = pv[i];
  if (to_backup) {
    s.z = s.x;
  } else {
    s.x = s.z;
    pq[i] = s.x / (s.w * s.w);
  }
  pv[i] = s;
}

// Algorithm 2 after the correction: new velocity and position, validity,
// and the request of a smaller step for a particle whose speed or
// acceleration no longer fits its region (its block and the 26 around it).
__global__ void k_pci_integrate(DevParams p, float4 *__restrict__ P, float4 *__restrict__ V,
                                float4 *__restrict__ A, uint32_t *__restrict__ M,
                                const float4 *__restrict__ fvg, const float4 *__restrict__ fp,
                                const float4 *__restrict__ pv, const float *__restrict__ pq,
                                const uint32_t *__restrict__ key, uint32_t *__restrict__ dem,
                                int major_len) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = i < p.n;  // every lane reaches the wave-wide requests below
  uint32_t need = kNoLevel, b = 0u;
  if (live) {
    const float dt = p.dt_base;
    const float4 a0 = fvg[i], a1 = fp[i];
    const float ax = a0.x + a1.x, ay = a0.y + a1.y, az = a0.z + a1.z;
    float4 v = V[i], x = P[i];
    v.x += dt * ax;
    v.y += dt * ay;
    v.z += dt * az;
    x.x += dt * v.x;
    x.y += dt * v.y;
    x.z += dt * v.z;
    x.w = pv[i].w;
    v.w = pq[i];
    P[i] = x;
    V[i] = v;
    A[i] = make_float4(ax, ay, az, 0.0f);
    const uint32_t m = M[i];
    const uint32_t l = meta_level(m);
    int32_t val = meta_validity(m) - 1;
    uint32_t comp = 0u;
    if (val <= 0) {
      comp = 1u;
      val = region_validity((int)l, major_len);
    }
    M[i] = meta_pack(l, comp, 0u, val);
    if (p.mode == RTS_MODE_RTS) {
      const float v2 = norm2_exact(v.x, v.y, v.z), a2 = norm2_exact(ax, ay, az);
      uint32_t lv = 0;
      while ((int)lv + 1 <= p.lmax && v2 <= p.TV[lv + 1] && a2 <= p.TA[lv + 1]) ++lv;
      if (lv < l) {
        need = lv;
        b = key[i];
      }
    }
  }
  // Requests of the wave, one lane per distinct block with the smallest level
  // its particles ask for (particles arrive in block order, so a burst of
  // requests costs few atomics).
  unsigned long long todo = __ballot(need != kNoLevel);
  const int lane = threadIdx.x & 63;
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const uint32_t lb = (uint32_t)__shfl((int)b, leader, 64);
    const bool mine = need != kNoLevel && b == lb;
    const uint32_t lvl = wave_min_u32(mine ? need : kNoLevel);
    if (lane == leader) {
      const int3 c = coords_of(p, lb);
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx) {
            const int bx = c.x + dx, by = c.y + dy, bz = c.z + dz;
            if (bx < 0 || by < 0 || bz < 0 || bx >= p.nc[0] || by >= p.nc[1] || bz >= p.nc[2])
              continue;
            atomicMin(&dem[(uint32_t)(bx + p.nc[0] * (by + p.nc[1] * bz))], lvl);
          }
    }
    if (mine) need = kNoLevel;
    todo = __ballot(need != kNoLevel);
  }
}

// Occupied blocks take the smallest requested level; every request is
// cleared for the next minor step.
__global__ void k_pci_demote_blocks(DevParams p, uint8_t *__restrict__ lvl,
                                    uint32_t *__restrict__ dem) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= p.nb) return;
  const uint32_t r = dem[b];
  if (r == kNoLevel) return;
  const uint8_t l = lvl[b];
  if (l != kEmpty && r < (uint32_t)l) lvl[b] = (uint8_t)r;
  dem[b] = kNoLevel;
}
__global__ void k_pci_demote_particles(DevParams p, const uint32_t *__restrict__ key,
                                       const uint8_t *__restrict__ lvl, uint32_t *__restrict__ M,
                                       int major_len) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  const uint32_t l = lvl[key[i]];
  const uint32_t m = M[i];
  if (l < meta_level(m)) M[i] = meta_pack(l, 1u, 0u, region_validity((int)l, major_len));
}

// Row view of the lists (debug): out[i * cap + k] = entry k of particle i.
__global__ void k_pci_lists_rows(DevParams p, const uint32_t *__restrict__ nbr,
                                 const uint32_t *__restrict__ nnb, uint32_t *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  const uint32_t cnt = min(nnb[i], (uint32_t)p.nbr_cap);
  for (uint32_t k = 0; k < (uint32_t)p.nbr_cap; ++k)
    out[(size_t)i * (size_t)p.nbr_cap + k] =
        k < cnt ? nbr[list_word((uint32_t)i, k, (size_t)p.ncap)] : 0u;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {
unsigned grid_of(int64_t n, int t) { return (unsigned)((n + t - 1) / t > 0 ? (n + t - 1) / t : 1); }
}  // namespace

void launch_pci_dilate(const DevParams &p, const DevPtrs &d, const uint8_t *src, uint8_t *dst,
                       int level, int layers, hipStream_t st) {
  const unsigned g = grid_of(p.nb, 256);
  hipLaunchKernelGGL(k_pci_dil_x, dim3(g), dim3(256), 0, st, p, src, d.DIL1, level, layers);
  hipLaunchKernelGGL(k_pci_dil_y, dim3(g), dim3(256), 0, st, p, d.DIL1, d.DIL2, layers);
  hipLaunchKernelGGL(k_pci_dil_z, dim3(g), dim3(256), 0, st, p, d.DIL2, src, dst, level, layers);
}
void launch_pci_major_flags(const DevParams &p, const DevPtrs &d, int cur, int major_len,
                            hipStream_t st) {
  if (p.n == 0) return;
  hipLaunchKernelGGL(k_pci_major_flags, dim3(grid_of(p.n, 256)), dim3(256), 0, st, p, d.KEY,
                     d.LVL, d.M[cur], major_len);
}
void launch_pci_observed(const DevParams &p, const DevPtrs &d, hipStream_t st) {
  hipLaunchKernelGGL(k_pci_observed, dim3(grid_of(p.nb, 256)), dim3(256), 0, st, p, d.OCC, d.LVL,
                     d.OB, d.S);
}
void launch_pci_lists(const DevParams &p, const DevPtrs &d, int cur, hipStream_t st) {
  if (p.n == 0) return;
  hipLaunchKernelGGL(k_pci_lists, dim3(grid_of((int64_t)p.n * kPciSub, 256)), dim3(256), 0, st,
                     p, d.P[cur], d.M[cur], d.KEY, d.CELL_START, d.WP, d.WCELL_START, d.NBRL,
                     d.NNB, d.ID[cur], d.S);
  hipLaunchKernelGGL(k_pci_nonpressure, dim3(grid_of(p.n, 256)), dim3(256), 0, st, p, d.P[cur],
                     d.V[cur], d.M[cur], d.NBRL, d.NNB, d.WP, d.FVG);
}
void launch_pci_reset(const DevParams &p, const DevPtrs &d, hipStream_t st) {
  const int64_t m = p.n > p.nb ? p.n : p.nb;
  hipLaunchKernelGGL(k_pci_reset, dim3(grid_of(m, 256)), dim3(256), 0, st, p, d.PV, d.FP, d.PQ,
                     d.SE, d.NEARSE);
}
void launch_pci_predict(const DevParams &p, const DevPtrs &d, int cur, hipStream_t st) {
  if (p.n == 0) return;
  hipLaunchKernelGGL(k_pci_predict, dim3(grid_of(p.n, 256)), dim3(256), 0, st, p, d.P[cur],
                     d.V[cur], d.FVG, d.FP, d.PQ, d.XS);
}
void launch_pci_density(const DevParams &p, const DevPtrs &d, int cur, uint32_t turn,
                        hipStream_t st) {
  if (p.n == 0) return;
  hipLaunchKernelGGL(k_pci_density, dim3(grid_of(p.n, 256)), dim3(256), 0, st, p, d.XS, d.PV,
                     d.PQ, d.M[cur], d.KEY, d.OB, d.NEARSE, d.SE, d.NBRL, d.NNB, d.WP, turn);
}
void launch_pci_mark_se(const DevParams &p, const DevPtrs &d, hipStream_t st) {
  if (p.n == 0) return;
  hipLaunchKernelGGL(k_pci_mark_se, dim3(grid_of(p.n, 256)), dim3(256), 0, st, p, d.SE, d.KEY,
                     d.NEARSE);
}
void launch_pci_force(const DevParams &p, const DevPtrs &d, int cur, uint32_t turn,
                      hipStream_t st) {
  if (p.n == 0) return;
  hipLaunchKernelGGL(k_pci_force, dim3(grid_of(p.n, 256)), dim3(256), 0, st, p, d.XS,
                     d.M[cur], d.SE, d.NBRL, d.NNB, d.WP, d.FP, turn);
}
void launch_pci_errstats(const DevParams &p, const DevPtrs &d, int cur, int first,
                         hipStream_t st, bool motion) {
  hipLaunchKernelGGL(k_pci_errstats, dim3(kPciStatBlocks), dim3(256), 0, st, p, d.PV, d.M[cur],
                     motion ? d.V[cur] : nullptr, motion ? d.A[cur] : nullptr, d.PPART, d.PCI,
                     first);
}
void launch_pci_pressure_copy(const DevParams &p, const DevPtrs &d, int to_backup,
                              hipStream_t st) {
  if (p.n == 0) return;
  hipLaunchKernelGGL(k_pci_pressure_copy, dim3(grid_of(p.n, 256)), dim3(256), 0, st, p, d.PV,
                     d.PQ, to_backup);
}
void launch_pci_integrate(const DevParams &p, const DevPtrs &d, int cur, int major_len,
                          hipStream_t st) {
  if (p.n == 0) return;
  hipLaunchKernelGGL(k_pci_integrate, dim3(grid_of(p.n, 256)), dim3(256), 0, st, p, d.P[cur],
                     d.V[cur], d.A[cur], d.M[cur], d.FVG, d.FP, d.PV, d.PQ, d.KEY, d.DEM,
                     major_len);
}
void launch_pci_lists_rows(const DevParams &p, const DevPtrs &d, uint32_t *out, hipStream_t st) {
  if (p.n == 0) return;
  hipLaunchKernelGGL(k_pci_lists_rows, dim3(grid_of(p.n, 256)), dim3(256), 0, st, p, d.NBRL,
                     d.NNB, out);
}
void launch_pci_demote(const DevParams &p, const DevPtrs &d, int cur, int major_len,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_pci_demote_blocks, dim3(grid_of(p.nb, 256)), dim3(256), 0, st, p, d.LVL,
                     d.DEM);
  if (p.n > 0)
    hipLaunchKernelGGL(k_pci_demote_particles, dim3(grid_of(p.n, 256)), dim3(256), 0, st, p,
                       d.KEY, d.LVL, d.M[cur], major_len);
  launch_pci_observed(p, d, st);
}

}  // namespace rts
