// Internal declarations of the RTS HIP library: device parameter block,
// device buffer table, per-run counters and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rts.h"

namespace rts {

constexpr uint32_t kWallBit = 0x80000000u;
constexpr uint8_t kEmpty = 0xFF;      // level of a block holding no fluid
constexpr int kMaxLevels = RTS_MAX_LEVELS;
constexpr int kCellMax = 512;         // particles per block the sort can canonicalise
constexpr int kScanTile = 1024;       // elements per scan workgroup (256 threads x 4)

// Meta word of a particle: bits 0-3 level, 4 compute, 5-15 age (base steps
// since the last evaluation), 16-31 validity (int16).
__host__ __device__ inline uint32_t meta_pack(uint32_t level, uint32_t compute, uint32_t age,
                                              int32_t validity) {
  return (level & 0xFu) | ((compute & 1u) << 4) | ((age & 0x7FFu) << 5) |
         ((uint32_t)(uint16_t)(int16_t)validity << 16);
}
__host__ __device__ inline uint32_t meta_level(uint32_t m) { return m & 0xFu; }
__host__ __device__ inline uint32_t meta_compute(uint32_t m) { return (m >> 4) & 1u; }
__host__ __device__ inline uint32_t meta_age(uint32_t m) { return (m >> 5) & 0x7FFu; }
__host__ __device__ inline int32_t meta_validity(uint32_t m) { return (int32_t)(int16_t)(m >> 16); }

// Numbers every kernel needs, derived once on the host in double precision
// and rounded to float.
struct DevParams {
  int32_t n, ncap, nw;
  int32_t cand_cap;      // candidates per block (list entries are 16-bit candidate indices)
  int32_t nbr_stride;    // WCSPH list row: nbr_cap + 1 rounded up to a multiple of 64, + 64
  int32_t nc[3];
  int32_t nb;
  int32_t act_cap;       // entries per active-block list segment: ceil(nb / kActParts)
  float o[3];
  float inv_e, r2f;
  float h, inv_h, sigma, mass;
  float dmax[3];         // domain upper corner (particles beyond it are an error)
  float kms;             // m sigma / rho0
  float c_hi, c_lo;      // rho0 / (m sigma) - 1 split in two floats (density deviation)
  float cs_hi, cs_lo;    // rho0 / (m sigma), the same with the particle's own W(0) = 1 kept
  float B, rho0;
  float visc_num;        // 2 alpha h c0
  float visc_eps_h2;     // eps h^2
  float g[3];
  float dt_base;
  double dt_cfl;         // lambda_v r / c0 (adaptive comparator)
  double lf2r;           // lambda_f^2 r (adaptive comparator: dt^2 <= lf2r / |a|)
  int32_t lmax, mode, serna_correct, clamp_p;
  int32_t phase_align;   // validity runs to the next multiple of 2^level
  int32_t n_scenes;      // independent scenes in the particle set (1 unless batched)
  float TV[kMaxLevels], TA[kMaxLevels];
  // PCISPH
  int32_t solver;
  int32_t nbr_cap;       // list entries per particle (both solvers)
  int32_t two_ring_levels;  // regions (levels 0..k-1) whose lists search two block layers
  float support;         // kernel support r
  float r2l;             // list radius squared
  float delta;           // pressure per unit density excess
  float eta_half;        // S_e threshold: half the allowed compression
  float pci_nu;          // artificial viscosity alpha h c0 / rho0
  float w0m;             // m W(0), the self term of the density
};

// Reductions of one PCISPH correction iteration, read by the host.
struct DevPci {
  float errmax;          // max over particles of max(err, 0)
  uint32_t ticket;       // last-workgroup detection of the fold (back to 0 after it)
  double avg;            // mean over particles of max(err, 0)
  int32_t hist[4];       // particles per region
  int32_t ncomp;         // particles with the compute flag
  int32_t ncomp_first;   // the same at the first iteration of the minor step (lists built)
  float v2max, a2max;    // max |v|^2 and |a|^2 after the step (when asked for)
};
struct PciPart {
  float errmax;
  int32_t ncomp;
  double sum;
  int32_t hist[4];
  float v2max, a2max;
};
constexpr int kPciStatBlocks = 128;

// Control words.  Zeroed once when the context is created and never reset
// or restored afterwards: the scan epoch only grows, so look-back words left
// by an earlier scan can never be mistaken for the current one's.  The
// tickets and the active-block count restart at every step's first kernel.
struct DevCtrl {
  uint32_t epoch;
  uint32_t scan_ticket;
  uint32_t stats_ticket;
  uint32_t search_ticket;   // next entry of the active-block list (search + density)
  uint32_t force_ticket;    // next entry of the active-block list (forces)
  uint32_t pad[3];
};

// The active-block list is kActBuckets segments of act_cap entries, read in
// segment order.  A block appends to segment kActParts c + s: its size class
// c runs from 0 (more than 16 (kActClasses - 1) active particles) to
// kActClasses - 1 (at most 16), its part s is its position among the nocc
// occupied blocks in kActParts equal ranges.  The list thus hands out the
// blocks with the most work first and the smallest last, so that persistent
// workgroups taking blocks in list order finish close together, and the
// appends spread over kActBuckets counters.  A part holds at most
// ceil(nocc / kActParts) blocks, so act_cap = ceil(nb / kActParts) entries
// always suffice.
constexpr int kActBuckets = 256;
constexpr int kActClasses = 8;
constexpr int kActParts = kActBuckets / kActClasses;
// Segment r's length lives at ACTN[r kActnStride]: one counter per 256 bytes,
// so that appends to different segments do not queue on one cache line.
constexpr int kActnStride = 64;

// Counters kept on the device (part of the saved state).
struct DevScalars {
  uint32_t status;
  int32_t bad_index;         // caller index of the particle that raised status, or -1
  uint32_t n_act;            // active particles of the last step
  uint32_t n_occ;            // occupied blocks of the current grid
  uint32_t nbr_max;
  float err_last;            // last step's max compression error
  float err_run;
  float amax2;               // max |a|^2 over the last step's active particles
  int32_t hist[kMaxLevels];
  unsigned long long inter_last;
  unsigned long long cand_last;      // candidate pair tests of the last step
  unsigned long long active_total;
  unsigned long long inter_total;
  unsigned long long cand_total;
  long long step;
  double time;
  double dt_prev;            // length of the step that ended at this step's start
  double dt_next;            // length of this step (predictor)
};

// Per-workgroup partial of the per-step statistics reduction.
struct StatPart {
  unsigned long long act, inter, cand;
  uint32_t nmax;
  float err, amax2;
  int32_t hist[kMaxLevels];
};
constexpr int kStatBlocks = 64;

// WCSPH neighbour lists: row i of LIST (nbr_stride entries) holds the local
// candidate indices, within its block's candidate set, of particle i's
// neighbours and of i itself, ascending (the canonical order); NNB[i] counts
// the neighbours.  The force pass gives kSub lanes to
// each particle.
constexpr int kSub = 8;

// Per-scene counters of a batched context (rts_get_scene_stats): integer
// atomics and a max over non-negative float bits, so the result does not
// depend on the order of the updates.
struct SceneStat {
  unsigned long long inter;  // neighbour pairs of the scene's active particles
  uint32_t act;              // active particles
  uint32_t err_bits;         // max(compression, 0) as float bits
  int32_t hist[kMaxLevels];  // particles per level
};
constexpr int kMaxScenes = RTS_MAX_SCENES;

struct DevPtrs {
  float4 *P[2];      // x, y, z, rho
  float4 *V[2];      // vx, vy, vz, p / rho^2
  float4 *A[2];      // stored acceleration
  uint32_t *M[2];    // meta
  uint32_t *ID[2];   // caller index
  float4 *ANEW;      // acceleration evaluated this step
  float *PRES;       // pressure (last step's active particles)
  uint32_t *KEY;     // block of each sorted particle
  uint32_t *KEYOLD;  // block of each particle in the previous order
  uint32_t *RANK;    // arrival slot within its block (unordered)
  uint32_t *TMP;     // block-grouped previous indices, unordered within a block
  uint32_t *PERM;    // previous index of each sorted particle
  uint32_t *NNB;     // neighbour count per particle (last step's active ones)
  uint16_t *LIST;    // ncap x nbr_stride WCSPH neighbour lists (16-bit candidate indices)
  uint32_t *COUNT;   // nb, zero between sorts
  uint32_t *CELL_START;  // nb + 1
  uint32_t *OCC;     // occupied blocks, ascending
  uint4 *OCCR;       // the same blocks with their sorted range: key, first slot, end slot, 0
  uint32_t *ACT;     // blocks holding an active particle this step, kActBuckets segments
  uint32_t *ACTN;    // kActBuckets segment lengths (kActnStride apart), zero at every step's start
  uint8_t *LRAW, *LVL;   // block level before / after R_min
  uint4 *BLKU;       // per block: active, pairs, candidate tests, max count | n << 16
  float *BLKERR;     // per block: max compression error
  float *BLKAMAX;    // per block: max |a|^2 of active particles
  StatPart *PART;    // kStatBlocks partials
  float4 *WP;        // wall particles, sorted
  uint32_t *WID, *WCELL_START, *WKEY, *WRANK, *WTMP;
  unsigned long long *TILES;   // scan look-back words, counts
  unsigned long long *TILES2;  // scan look-back words, occupied blocks
  DevCtrl *CTRL;
  DevScalars *S;
  // PCISPH (one entry when the solver is WCSPH)
  float4 *XS;        // predicted position x*
  float4 *PV;        // pressure, relative density error, pressure backup, rho*
  float4 *FVG;       // gravity + viscosity acceleration
  float4 *FP;        // pressure acceleration
  float *PQ;         // p / rho*^2
  uint8_t *SE;       // member of S_e
  uint32_t *NBRL;    // nbr_cap x ncap neighbour lists in quads (entry k of i at word
                     // ((k/4) ncap + i) 4 + k%4)
  uint8_t *OB;       // per block: observed
  uint8_t *NEARSE;   // per block: holds or borders an S_e particle
  uint8_t *DIL1, *DIL2;  // per block: dilation masks
  uint8_t *DILT, *DILATED;  // per block: levels after the first / both dilations
  uint32_t *DEM;     // per block: smallest level requested this minor step
  PciPart *PPART;    // kPciStatBlocks partials
  DevPci *PCI;
  // scenes: caller index of each scene's first particle (n_scenes + 1
  // entries, the last = n) and their counters
  uint32_t *SCN_OFF;
  SceneStat *SCN_STAT;
};

// Launchers (rts_kernels.hip).  All enqueue on `st`.
void launch_key_hist(const DevParams &p, const DevPtrs &d, int cur, hipStream_t st);
void launch_scan(const DevParams &p, const DevPtrs &d, uint32_t *start, bool fluid,
                 hipStream_t st);
void launch_prep_scan(DevCtrl *ctrl, hipStream_t st);
void launch_scatter(const DevParams &p, const DevPtrs &d, hipStream_t st);
void launch_cell_gather(const DevParams &p, const DevPtrs &d, int cur, int grid, hipStream_t st);
void launch_rmin_flags(const DevParams &p, const DevPtrs &d, int cur, int do_flags, int grid,
                       hipStream_t st, const uint8_t *src = nullptr);
// threads: 256 or 512 per workgroup; lanes: 4 or 8 per particle
void launch_search_density(const DevParams &p, const DevPtrs &d, int cur, int grid, int threads,
                           hipStream_t st);
void launch_force(const DevParams &p, const DevPtrs &d, int cur, int grid, int lanes,
                  hipStream_t st);
void launch_step_stats(const DevParams &p, const DevPtrs &d, hipStream_t st);
void launch_debug_lists(const DevParams &p, const DevPtrs &d, int cur, uint32_t *out, uint32_t *out_n,
                        hipStream_t st);
void launch_correct_predict(const DevParams &p, const DevPtrs &d, int cur, hipStream_t st);
void launch_stats_correct_predict(const DevParams &p, const DevPtrs &d, int cur,
                                  hipStream_t st);
void launch_set_state(const DevParams &p, const DevPtrs &d, int cur, const float *pos,
                      const float *vel, hipStream_t st);
void launch_add_velocity(const DevParams &p, const DevPtrs &d, int cur, const float *dv,
                         hipStream_t st);
// Lattice column with SplitMix64 jitter into caller slots [first, first + cnt)
// of buffer 0, as rts_set_state leaves a particle (at rest, due at once).
struct LatticeSpec {
  int32_t counts[3];
  int32_t pad;
  double corner[3];
  double spacing, jitter;
  unsigned long long seed, first_draw;
};
void launch_init_lattice(const DevParams &p, const DevPtrs &d, uint32_t first, uint32_t cnt,
                         const LatticeSpec &L, hipStream_t st);
void launch_scene_stats(const DevParams &p, const DevPtrs &d, int cur, hipStream_t st);
// rts_get_state restricted to caller indices [lo, lo + cnt), written from 0
void launch_get_range(const DevParams &p, const DevPtrs &d, int cur, uint32_t lo, uint32_t cnt,
                      float *pos, float *vel, float *acc, float *rho, float *pres,
                      uint8_t *level, hipStream_t st);
void launch_get_state(const DevParams &p, const DevPtrs &d, int cur, float *pos, float *vel,
                      float *acc, float *rho, float *pres, uint8_t *level, hipStream_t st);
void launch_wall_sort(const DevParams &p, const DevPtrs &d, const float *pos, hipStream_t st);
void launch_reset_scalars(DevScalars *S, hipStream_t st);
// p must be 4-byte aligned
void launch_fill(void *p, uint8_t v, size_t bytes, hipStream_t st);

// PCISPH launchers (pcisph_kernels.hip)
void launch_pci_dilate(const DevParams &p, const DevPtrs &d, const uint8_t *src, uint8_t *dst,
                       int level, int layers, hipStream_t st);
void launch_pci_major_flags(const DevParams &p, const DevPtrs &d, int cur, int major_len,
                            hipStream_t st);
void launch_pci_observed(const DevParams &p, const DevPtrs &d, hipStream_t st);
void launch_pci_lists(const DevParams &p, const DevPtrs &d, int cur, hipStream_t st);
void launch_pci_reset(const DevParams &p, const DevPtrs &d, hipStream_t st);
void launch_pci_predict(const DevParams &p, const DevPtrs &d, int cur, hipStream_t st);
void launch_pci_density(const DevParams &p, const DevPtrs &d, int cur, uint32_t turn,
                        hipStream_t st);
void launch_pci_mark_se(const DevParams &p, const DevPtrs &d, hipStream_t st);
void launch_pci_force(const DevParams &p, const DevPtrs &d, int cur, uint32_t turn,
                      hipStream_t st);
void launch_pci_errstats(const DevParams &p, const DevPtrs &d, int cur, int first,
                         hipStream_t st, bool motion = false);
void launch_pci_pressure_copy(const DevParams &p, const DevPtrs &d, int to_backup,
                              hipStream_t st);
void launch_pci_integrate(const DevParams &p, const DevPtrs &d, int cur, int major_len,
                          hipStream_t st);
void launch_pci_demote(const DevParams &p, const DevPtrs &d, int cur, int major_len,
                       hipStream_t st);
void launch_pci_lists_rows(const DevParams &p, const DevPtrs &d, uint32_t *out, hipStream_t st);

// Differentiable substep launchers (diff_kernels.hip)
void launch_diff_planes_in(int n, const float *src, float4 *dst, hipStream_t st);
void launch_diff_planes_out(int n, const float4 *src, float *dst, hipStream_t st);
void launch_diff_zero(int n, float4 *a, double *b, double *c, hipStream_t st);
void launch_diff_setup(const DevParams &p, const DevPtrs &d, int n, int cap, float B,
                       const float4 *X, const float4 *V, uint32_t *L, uint32_t *nn, float *rho,
                       float *prs, float4 *XP, float4 *VR, int grid_wave, hipStream_t st);
void launch_diff_force_euler(const DevParams &p, const DevPtrs &d, int n, int cap, float dt,
                             float alpha, float hc0, const float4 *XP, const float4 *VR,
                             const uint32_t *L, const uint32_t *nn, float4 *Xn, float4 *Vn,
                             hipStream_t st);
void launch_diff_adjoint(const DevParams &p, const DevPtrs &d, int n, int cap, float dt, float B,
                         float alpha, float hc0, const float4 *X, const float4 *V,
                         const float *rho, const float *prs, const uint32_t *L,
                         const uint32_t *nn, float4 *XB, float4 *VB, float4 *AB, float4 *XR,
                         float4 *VP, float4 *XRB, double *BB, double *AA, hipStream_t st);
void launch_diff_reduce(int n, const double *BB, const double *AA, double *out, hipStream_t st);

}  // namespace rts
