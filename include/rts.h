/*
 * rts.h -- C ABI of the MI355X regional time stepping (RTS) SPH library.
 *
 * Method: Goswami & Batty, "Asynchronous Liquids: Regional Time Stepping for
 * Faster SPH and PCISPH".  The fluid domain is cut into blocks whose edge is
 * at least the kernel support (Section 3); each block gets a time step from
 * the speed and acceleration of its particles (Section 3.1, Eq. 1-3), and
 * only particles whose step ends re-evaluate density and forces, with the
 * predictor-corrector of Serna et al. keeping everyone in step (Section 4,
 * Algorithm 1).
 *
 * Conventions for every entry point
 *   - Pointers named d_* are device memory owned by the caller and borrowed
 *     only for the duration of the call (or, for the workspace, until
 *     rts_destroy).  Pointers named h_* are host memory.
 *   - Vector arrays passed in or out are structure-of-arrays planes of
 *     float32: x[0..n), then y[0..n), then z[0..n).
 *   - Per-particle outputs are in the caller's original particle order
 *     (the order given to rts_set_state).
 *   - Work is enqueued on the HIP stream given to rts_create and calls
 *     return before it finishes, except rts_sync, rts_assign_levels and the
 *     getters that return host values, which wait for the stream.
 *   - Every call returns an rts_status.  rts_last_error() gives a message.
 *     Invalid arguments are rejected before any device work is enqueued.
 *     After RTS_E_NUMERICAL or RTS_E_CAPACITY is reported by rts_sync the
 *     context stays valid, but rts_advance returns RTS_E_STATE until the
 *     state is replaced by rts_set_state or rts_load_state.
 *   - One context per host thread; contexts are independent.
 */
#ifndef RTS_H
#define RTS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RTS_OK = 0,
  RTS_E_INVALID = 1,     /* bad argument or configuration */
  RTS_E_CAPACITY = 2,    /* neighbour list, block population or workspace too small */
  RTS_E_DEVICE = 3,      /* a HIP runtime call failed */
  RTS_E_NUMERICAL = 4,   /* a particle became non-finite or left the domain */
  RTS_E_STATE = 5,       /* call not allowed in the current state */
  RTS_E_UNSUPPORTED = 6  /* configuration value this build does not implement */
} rts_status;

typedef enum { RTS_WCSPH = 0, RTS_PCISPH = 1 } rts_solver;

/* RTS: Algorithm 1 with block levels.  GLOBAL_FIXED: the same loop with
 * every block at level 0.  GLOBAL_ADAPTIVE: every particle active each step,
 * step length min(lambda_v r / c0, lambda_f sqrt(r / max|a|)). */
typedef enum { RTS_MODE_RTS = 0, RTS_MODE_GLOBAL_FIXED = 1, RTS_MODE_GLOBAL_ADAPTIVE = 2 } rts_mode;

#define RTS_MAX_LEVELS 8
#define RTS_DEBUG_NBR_ROW 1024  /* row width of the RTS_DBG_NBR view */

/* Run configuration.  SI units, double precision so that derived float
 * thresholds are rounded once from the exact configured values.
 * rts_default_config fills every field. */
typedef struct rts_config {
  int32_t solver;        /* rts_solver */
  int32_t mode;          /* rts_mode */
  int32_t n_levels;      /* number of block levels; level l steps 2^l base steps (<= 8) */
  int32_t level_cap;     /* highest level a block may take */
  int32_t clamp_p;       /* clamp pressure at zero */
  int32_t serna_correct; /* 1: apply the predictor-corrector correction (Section 4.1) */
  int32_t cand_cap;      /* neighbour candidates per block (27 blocks + walls) that the 16-bit
                            entries of the WCSPH lists can index; multiple of 256, <= 65536 */
  int32_t use_graph;     /* 1: replay each base step as a captured HIP graph */
  double spacing;         /* initial particle spacing s */
  double h;               /* smoothing length of the cubic spline (support 2h) */
  double support;         /* kernel support radius, 2h */
  double block_edge;      /* block edge, >= support */
  double r_crit;          /* length r of Eq. 1-3 (<= 0: support) */
  double rho0;            /* rest density */
  double mass;            /* particle mass (<= 0: rho0 / lattice sum of W) */
  double c0;              /* speed of sound */
  double gamma;           /* Tait exponent (this build: 7) */
  double B;               /* Tait stiffness (<= 0: rho0 c0^2 / gamma) */
  double visc_alpha;      /* artificial viscosity alpha */
  double visc_eps;        /* viscosity regulariser, times h^2 */
  double gravity[3];
  double domain_min[3];   /* block grid covers [domain_min, domain_max] */
  double domain_max[3];
  double dt_base;         /* base step (<= 0: lambda_v r_crit / c0, Eq. 1) */
  double lambda_v;        /* Eq. 1 coefficient (paper: <= 0.4) */
  double lambda_f;        /* Eq. 2 coefficient (paper: <= 0.25) */
  double alpha_rts;       /* Eq. 3 alpha (paper: 0.4 WCSPH, 1 PCISPH) */
  double beta2;           /* beta_2 of Eq. 3 (paper: 0.4) */
  double beta_ratio;      /* beta_{n+1} / beta_n (paper: 0.2) */
  /* PCISPH with regional iteration counts (Section 5, Algorithms 2-3).
   * Regions R_1..R_4 are block levels 0..3; region n steps n base steps in
   * Eq. 2-3 (Eq. 1 is not applied).  One rts_advance step is one minor
   * step of length dt_base; a major step is n_minor minor steps. */
  int32_t n_minor;        /* minor steps per major step (paper: 4) */
  int32_t it_min;         /* correction iterations per minor step, at least (3) */
  int32_t it_max;         /* ... and at most (50) */
  int32_t expand_layers;  /* regions 1 and 2 grow by this many block layers (4) */
  int32_t local_fail;     /* local iterations before reverting to global ones (3); a
                             minor step runs at most one local phase */
  int32_t global_limit;   /* global iterations in one minor step that end the major step (6) */
  int32_t short_majors;   /* clean major steps before the long major step returns (10) */
  int32_t nbr_cap;        /* neighbour-list entries per particle, in [8, 4096] (both solvers;
                             a particle with more neighbours fails the step with
                             RTS_E_CAPACITY; default 512) */
  int32_t two_ring_levels;/* regions whose lists search two block layers (paper: 1, region 1;
                             2 adds region 2, the variant of the paper's comparison figure) */
  int32_t pci_adapt_dt;   /* 1: adaptive base step between major steps (RTS mode; see below) */
  double eta;             /* allowed maximum compression (paper: 1 %) */
  double eta_T;           /* average compression above which extra iterations are global */
  double delta;           /* pressure coefficient (<= 0: from the full rest-lattice
                             neighbourhood, standard PCISPH) */
  double r_list;          /* neighbour-list radius (<= 0: block_edge, the 1.1 r grid) */
  /* Adaptive base step of regional PCISPH (the paper's conclusions suggest
   * combining the method with global adaptive stepping).  dt_base is the
   * first major step's base step.  After each major step the next one's is
   *   dt * pci_shrink  if a minor step ran more than global_limit global
   *                    iterations or more than pci_shrink_iters in all,
   *   dt * pci_grow    else if no minor step ran more than pci_grow_iters,
   *   dt               otherwise,
   * capped by pci_dt_max and by Eq. 3 with beta_2 and Eq. 2 for the fastest
   * particle (alpha beta_2 r / V_max, lambda_f sqrt(r / A_max)), and
   * raised to pci_dt_min.  A minor step whose correction still exceeds eta
   * after it_max iterations rolls its major step back to the state the
   * major step started from and restarts it with max(dt / 2, pci_dt_min),
   * as long as dt is above pci_dt_min; rts_advance counts accepted minor
   * steps.  Needs delta <= 0 (delta
   * follows the step). */
  int32_t pci_grow_iters; /* (<= 0: it_min) */
  int32_t pci_shrink_iters; /* (<= 0: it_min) */
  double pci_dt_min;      /* (<= 0: dt_base / 4) */
  double pci_dt_max;      /* (<= 0: 4 dt_base) */
  double pci_grow;        /* >= 1 (1.02) */
  double pci_shrink;      /* in (0, 1] (0.95) */
  /* WCSPH block levels (Algorithm 1).  0: a particle that takes level l
   * (its validity ran out, or its block's level changed) is next due 2^l
   * base steps later, as Algorithm 1 prints it.  1 (default): it is next
   * due at the next base step that is a multiple of 2^l, so all particles of
   * a level update on the same steps and a block's particles stay in phase;
   * steps only get shorter (at most 2^l base steps, as before), and the
   * blocks with work in a step are fewer. */
  int32_t phase_align;
  int32_t pad_;
} rts_config;

/* Per-run counters, filled by rts_sync. */
typedef struct rts_stats {
  int64_t step;                      /* base steps taken */
  double time;                       /* simulated time */
  double dt_last;                    /* length of the last step */
  int64_t active_last;               /* particles active in the last step */
  int64_t inter_last;                /* neighbour pairs of active particles in the last step */
  int64_t active_total;              /* sum over steps of active particles */
  int64_t inter_total;               /* sum over steps of neighbour pairs evaluated */
  int64_t cand_total;                /* sum over steps of candidate pair tests in the search */
  float err_max_last;                /* max over particles of max(rho - rho0, 0) / rho0, last step */
  float err_max_run;                 /* the same, max over all steps */
  int32_t level_hist[RTS_MAX_LEVELS];/* particles per level after the last step's flags */
  int32_t nbr_max;                   /* largest neighbour count seen */
  int32_t status;                    /* device status (rts_status) */
  int32_t bad_index;                 /* particle (caller order) that raised the status, or -1 */
  /* PCISPH, last minor step */
  int32_t pci_iters;                 /* correction iterations */
  int32_t pci_global_iters;          /* of which with the schedule (global) */
  int32_t pci_resets;                /* restarts of the schedule (average error too high,
                                        or any extra iteration after a failed local phase) */
  int32_t pci_reverts;               /* local phases abandoned, pressure restored */
  int32_t pci_early_end;             /* 1: the major step ended early after this step */
  int32_t pci_lists;                 /* neighbour lists rebuilt */
  int32_t pci_major_len;             /* current major-step length in minor steps */
  int32_t pci_minor_in_major;        /* minor steps done in the current major step */
  double pci_errmax;                 /* max compression after the last iteration */
  double pci_avg;                    /* mean compression after the last iteration */
  int64_t pci_iters_total;           /* iterations summed over all minor steps, rolled-back
                                        ones included */
  int32_t pci_rollbacks;             /* major steps rolled back (adaptive base step) */
  int32_t pci_pad;
  double pci_dt_next;                /* base step of the next minor step */
} rts_stats;

typedef struct rts_ctx rts_ctx;

/* Fills *cfg with the defaults (Section 3.1 constants, cubic spline h = 2s). */
void rts_default_config(rts_config *cfg);

/* Device workspace bytes for up to n_fluid_max fluid and n_wall_max wall
 * particles under cfg.  Returns RTS_E_INVALID for a bad configuration. */
rts_status rts_workspace_size(const rts_config *cfg, int64_t n_fluid_max, int64_t n_wall_max,
                              size_t *bytes);

/* Creates a context on the current HIP device.  d_workspace: caller device
 * memory of at least rts_workspace_size bytes, 256-byte aligned, kept alive
 * until rts_destroy.  hip_stream: the hipStream_t to enqueue on (NULL: the
 * null stream).  The context is empty until rts_set_state. */
rts_status rts_create(const rts_config *cfg, int64_t n_fluid_max, int64_t n_wall_max,
                      void *d_workspace, size_t bytes, void *hip_stream, rts_ctx **out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): rts_create with
 * the library's own workspace instead of a caller buffer.  The workspace is
 * a static device array of RTS_STATIC_WORKSPACE_BYTES per device, reserved
 * when the library is loaded and held until the process ends; its address
 * on the current device is looked up on the first call there.  The call
 * allocates no device memory and launches only kernels on hip_stream (it
 * clears the counters the run needs at zero; the array keeps whatever the
 * previous context there left).  The context behaves exactly like one from
 * rts_create; to keep rts_advance free of allocations too, set use_graph = 0
 * (graph instantiation allocates).
 *   RTS_E_CAPACITY: rts_workspace_size(cfg, n_fluid_max, n_wall_max) exceeds
 *                   RTS_STATIC_WORKSPACE_BYTES;
 *   RTS_E_STATE:    another live context on this device already uses the
 *                   array (one at a time per device; rts_destroy frees it);
 *   RTS_E_DEVICE:   no current device, or its array could not be located;
 *   RTS_E_INVALID:  as rts_create.
 * Work on the array from different host threads is serialised only at
 * create / destroy: calls on one context must not overlap in time. */
#define RTS_STATIC_WORKSPACE_BYTES (32u << 20)
rts_status rts_create_static(const rts_config *cfg, int64_t n_fluid_max, int64_t n_wall_max,
                             void *hip_stream, rts_ctx **out);

/* Batched scenes: independent scenes of n_per_scene[s] particles each in
 * one context (the benchmark spec's batched configuration), stepped together by
 * every rts_advance; scene s holds caller indices [first_s, first_s + n_s)
 * with first_s = n_0 + ... + n_{s-1}.  The scenes must be placed apart in
 * space (their kernel supports disjoint, walls included) and share the
 * configuration, so one sound speed and one base step (Eq. 1) hold for all.
 * d_workspace: at least rts_workspace_size(cfg, sum of n_per_scene,
 * n_wall_max) bytes.  WCSPH only (RTS_E_UNSUPPORTED otherwise); 1 <=
 * n_scenes <= RTS_MAX_SCENES.  rts_set_state then takes exactly the summed
 * count; rts_init_dam_break fills scenes on the device. */
#define RTS_MAX_SCENES 4096
rts_status rts_create_batch(const rts_config *cfg, int32_t n_scenes, const int64_t *h_n_per_scene,
                            int64_t n_wall_max, void *d_workspace, size_t bytes,
                            void *hip_stream, rts_ctx **out);

/* Releases the host context and its graphs.  The workspace stays the caller's
 * (a static-workspace context releases its claim on the device's array). */
void rts_destroy(rts_ctx *ctx);

/* Static wall particles (boundary; Section 6 uses static boundary particles).
 * d_pos: 3*nw floats (planes).  Sorted into the block grid once. */
rts_status rts_set_walls(rts_ctx *ctx, const float *d_pos, int64_t nw);

/* Replaces the fluid state: n particles, d_pos and d_vel 3*n floats each.
 * Accelerations start at zero and every particle starts with validity 0,
 * so the first step evaluates all of them (Algorithm 1 initialisation). */
rts_status rts_set_state(rts_ctx *ctx, const float *d_pos, const float *d_vel, int64_t n);

/* Scene initialisation on the device (the problem statement's "init
 * scene"), for contexts from rts_create_batch: writes a lattice column of
 * counts[0] x counts[1] x counts[2] particles (x fastest) into scene `scene`
 * from its particle `first` on, at h_corner + (i + 1/2) spacing per axis
 * plus a uniform jitter in [-jitter, jitter): u = (SplitMix64(seed) output
 * number 3 (first_draw + k) + axis, top 24 bits) / 2^24, offset
 * jitter (2u - 1), all in double precision with each operation rounded on
 * its own, then rounded to float; particles at rest, due at once, as after
 * rts_set_state.  A scene may take several columns (e.g. the two of a
 * double dam break); the context has a state once every particle of every
 * scene is written.  The first call after a step (or any call that sorted
 * the particles) starts a new run: every scene must be written again.
 * RTS_E_INVALID: bad scene, negative counts, a column past the scene's
 * end; RTS_E_STATE: a context from rts_create.  Asynchronous. */
rts_status rts_init_dam_break(rts_ctx *ctx, int32_t scene, int64_t first, const int32_t *h_counts,
                              const double *h_corner, double spacing, double jitter,
                              uint64_t seed, uint64_t first_draw);

/* External impulse: adds d_dv (planes, 3*n floats, caller order) to the
 * particles' velocities and changes nothing else: levels, validity, ages and
 * stored accelerations stay.  The next base step's block maxima see the new
 * speeds, so a block that now needs a smaller step takes it and its
 * particles that were in the middle of a longer step are pre-empted
 * (Section 4.2, pre-emption; Algorithm 1: a particle whose parent block has a
 * different step recomputes).  PCISPH: the next minor step's smaller-step
 * check sees them; with the adaptive base step a roll-back of the current
 * major step discards the impulse.  n must equal the particle count given
 * to rts_set_state (else RTS_E_INVALID); RTS_E_STATE before any state.
 * Asynchronous; d_dv must stay valid until the stream reaches the call. */
rts_status rts_add_velocity(rts_ctx *ctx, const float *d_dv, int64_t n);

/* Region determination only (Section 3.1 and R_min of Section 4.2): rebuilds
 * the block grid, takes block maxima and levels and smooths them, without
 * touching particle flags or physics.  h_level_hist[n_levels]: number of
 * occupied blocks per level.  Waits for the stream.
 * PCISPH: the set-up of a major step (Algorithm 2): grid of edge block_edge,
 * regions from Eq. 2-3, dilation of regions 1 and 2, R_min, observed blocks,
 * particle regions and flags; the next rts_advance continues that major
 * step instead of starting one. */
rts_status rts_assign_levels(rts_ctx *ctx, int32_t *h_level_hist);

/* Advances n_steps base steps of Algorithm 1 (or of the global comparator
 * chosen by cfg.mode).  Asynchronous.
 * PCISPH: n_steps minor steps of Algorithm 2 with the density correction of
 * Algorithm 3; each correction iteration waits for the stream to read the
 * error reductions that decide the next one, so the call returns after the
 * work is done.  RTS_MODE_GLOBAL_FIXED runs standard PCISPH (grid and lists
 * every step, every particle in every iteration) as the comparator. */
rts_status rts_advance(rts_ctx *ctx, int32_t n_steps);

/* Waits for the stream and copies the counters to *h_out (may be NULL).
 * Returns the device status. */
rts_status rts_sync(rts_ctx *ctx, rts_stats *h_out);

/* Copies the state out in caller order.  Any pointer may be NULL.
 * d_pos, d_vel, d_acc: 3*n floats; d_rho, d_p: n floats; d_level: n bytes. */
rts_status rts_get_state(rts_ctx *ctx, float *d_pos, float *d_vel, float *d_acc, float *d_rho,
                         float *d_p, uint8_t *d_level);

/* Per-scene counters after the last step (any context; one scene unless
 * batched): caller index of the scene's first particle, its particle
 * count, particles active in the last step and their neighbour pairs, the
 * maximum compression max(rho - rho0, 0) / rho0 of the scene's stored
 * densities, and particles per level.  h_out[n_scenes]; n_scenes must equal
 * the context's.  Waits for the stream. */
typedef struct rts_scene_stats {
  int64_t first;
  int64_t n;
  int64_t active_last;
  int64_t inter_last;
  float err_max_last;
  int32_t level_hist[RTS_MAX_LEVELS];
  int32_t pad;
} rts_scene_stats;
rts_status rts_get_scene_stats(rts_ctx *ctx, rts_scene_stats *h_out, int32_t n_scenes);

/* rts_get_state for one scene: its particles in caller order, from slot 0
 * (3 * n_s floats per vector plane set, n_s per scalar).  Asynchronous. */
rts_status rts_get_scene_state(rts_ctx *ctx, int32_t scene, float *d_pos, float *d_vel,
                               float *d_acc, float *d_rho, float *d_p, uint8_t *d_level);

/* Saves / restores the complete state and counters, so that a restored run
 * continues bit for bit.  d_buf: device memory of at least rts_state_bytes.
 * WCSPH: the particle state (positions, velocities, accelerations, levels,
 * validity, ages, densities, pressures, caller ids) and the counters; it
 * loads into any context of the same grid with room for the particles.
 * PCISPH: an image of the context's whole workspace (both sort buffers, the
 * major step's grid, regions, observed blocks, lists, non-pressure
 * accelerations, errors) and the correction loop's host counters (position
 * in the major step, major-step length, clean major steps, step count,
 * simulated time, base step, roll-back point), taken at any minor step; it
 * loads only into a context created with the same configuration and
 * capacities (else RTS_E_INVALID). */
rts_status rts_state_bytes(rts_ctx *ctx, size_t *bytes);
rts_status rts_save_state(rts_ctx *ctx, void *d_buf, size_t cap);
rts_status rts_load_state(rts_ctx *ctx, const void *d_buf, size_t len);

/* Debug views of internal buffers, copied raw to d_out (device).  *n_out
 * receives the element count.  Layouts:
 *   RTS_DBG_POS/VEL/ACC/ACC_NEW: float4 per particle, sorted order
 *   RTS_DBG_META: uint32 per particle (bits 0-3 level, 4 compute, 5-15 age,
 *                 16-31 validity as int16), sorted order
 *   RTS_DBG_ID: caller index of each sorted particle
 *   RTS_DBG_KEY: block key of each sorted particle
 *   RTS_DBG_PERM: previous sorted position of each sorted particle
 *   RTS_DBG_CELL_START: nblocks + 1 uint32
 *   RTS_DBG_BLK_LEVEL_RAW / BLK_LEVEL: uint8 per block, before / after R_min
 *   RTS_DBG_NNB: uint32 per particle: neighbour count (last step's active)
 *   RTS_DBG_NBR: n x RTS_DEBUG_NBR_ROW uint32, row i = canonical neighbour
 *                 list of sorted particle i (ascending sorted index, then walls
 *                 as wall sorted index | 0x80000000), followed by n uint32 list
 *                 lengths; rows of particles inactive in the last step are empty
 *   RTS_DBG_PRESSURE: float per sorted slot, valid for the last step's active
 *                 particles only
 *   RTS_DBG_PRE_POS/VEL/ACC/META/ID: the arrays as they were before the last
 *                 step's sort (the step's input), in their previous order
 *   RTS_DBG_WALL_POS: float4 per wall particle, sorted; RTS_DBG_WALL_ID:
 *                 caller index of each sorted wall; RTS_DBG_WALL_CELL_START
 *   RTS_DBG_OCCUPIED: ascending keys of the blocks holding fluid
 *   RTS_DBG_BLK_STATS: uint32 x 4 per block, valid for occupied blocks: active
 *                 particles, neighbour pairs, candidate tests, and max neighbour
 *                 count | particles << 16, of the last step. */
typedef enum {
  RTS_DBG_POS = 0, RTS_DBG_VEL, RTS_DBG_ACC, RTS_DBG_ACC_NEW, RTS_DBG_META, RTS_DBG_ID,
  RTS_DBG_KEY, RTS_DBG_PERM, RTS_DBG_CELL_START, RTS_DBG_BLK_LEVEL_RAW, RTS_DBG_BLK_LEVEL,
  RTS_DBG_NNB, RTS_DBG_NBR, RTS_DBG_PRESSURE, RTS_DBG_PRE_POS, RTS_DBG_PRE_VEL,
  RTS_DBG_PRE_ACC, RTS_DBG_PRE_META, RTS_DBG_PRE_ID, RTS_DBG_WALL_POS, RTS_DBG_WALL_ID,
  RTS_DBG_WALL_CELL_START, RTS_DBG_OCCUPIED, RTS_DBG_BLK_STATS,
  /* PCISPH (block order of the current major step) */
  RTS_DBG_PCI_XS,        /* float4: predicted position x*, p / rho*^2 */
  RTS_DBG_PCI_PV,        /* float4: pressure, relative density error, pressure backup, rho* */
  RTS_DBG_PCI_FVG,       /* float4: non-pressure acceleration (gravity + viscosity), 0 */
  RTS_DBG_PCI_FP,        /* float4: pressure acceleration, 0 */
  RTS_DBG_PCI_SE,        /* uint8 per particle: member of S_e */
  RTS_DBG_PCI_OB,        /* uint8 per block: observed (borders a smaller region) */
  RTS_DBG_PCI_DILATED,   /* uint8 per block: levels after dilation, before R_min */
  RTS_DBG_PCI_LISTS,     /* uint32: n rows of nbr_cap entries (fluid sorted index,
                            walls | 0x80000000), then the n counts */
  RTS_DBG_COUNT_
} rts_debug_what;
rts_status rts_debug_get(rts_ctx *ctx, int32_t what, void *d_out, size_t cap_bytes, size_t *n_out);

/* Grid and derived numbers: nc[3], nblocks, particle mass, Tait B, base step. */
rts_status rts_grid_info(rts_ctx *ctx, int32_t *h_nc3, int64_t *h_nblocks, double *h_mass,
                         double *h_B, double *h_dt_base);

/* Timing aid: advances n_steps base steps like rts_advance, but launches the
 * kernels one by one with a HIP event between consecutive kernels on the
 * context's stream, and adds each kernel's time in milliseconds to
 * h_ms[0..RTS_PROF_COUNT) in the order of rts_prof_kernel.  Waits for the
 * stream.  The simulation result is identical to rts_advance.  (With a fixed
 * base step rts_advance runs the statistics, the corrector-predictor and the
 * next step's binning as one launch; here they are timed apart.) */
typedef enum {
  RTS_PROF_KEY_HIST = 0, RTS_PROF_SCAN, RTS_PROF_SCATTER, RTS_PROF_CELL_GATHER,
  RTS_PROF_RMIN_FLAGS, RTS_PROF_SEARCH_DENSITY, RTS_PROF_FORCE, RTS_PROF_STEP_STATS,
  RTS_PROF_CORRECT_PREDICT, RTS_PROF_COUNT
} rts_prof_kernel;
rts_status rts_profile_advance(rts_ctx *ctx, int32_t n_steps, double *h_ms);

/* Launch shape of the base step: workgroups of the one-wave-per-block
 * kernels, of the search + density kernel and of the force kernel. */
typedef struct rts_tune {
  int32_t grid_wave;      /* workgroups of the one-wave-per-block kernels */
  int32_t grid_search;    /* workgroups of the search / density kernel */
  int32_t grid_force;     /* workgroups of the force kernel */
  int32_t search_threads; /* threads per search workgroup: 256 or 512 */
  int32_t force_threads;  /* threads per force workgroup: 512 */
  int32_t force_lanes;    /* lanes sharing one particle in the force kernel: 4 or 8 */
  int32_t candidates;     /* shapes timed by rts_autotune */
  int32_t pad_;
  double ms_per_step;     /* replay time of the chosen shape */
} rts_tune;

/* Times `steps` base steps (WCSPH) under candidate launch shapes from the
 * current state and keeps the fastest, one kernel group at a time: the grid
 * of the one-wave-per-block kernels, then the search kernel's workgroup
 * size and count, then the force kernel's lanes per particle and workgroup
 * count.  The state is saved to d_scratch (at least rts_state_bytes) before
 * and restored after every candidate, so the run continues exactly as if no
 * tuning had happened: no launch shape changes any result (the force sums a
 * particle's terms in the same fixed order whatever its lanes).  Waits for
 * the stream. */
rts_status rts_autotune(rts_ctx *ctx, int32_t steps, void *d_scratch, size_t scratch_bytes,
                        rts_tune *h_out);
/* Current launch shape (h_out->candidates = 0, ms_per_step = 0 until tuned). */
rts_status rts_get_tune(rts_ctx *ctx, rts_tune *h_out);
/* Sets the launch shape (grids >= 1, the sizes above; candidates and
 * ms_per_step are ignored), e.g. one tuned before on the same scene.
 * RTS_E_INVALID for a shape out of range. */
rts_status rts_set_tune(rts_ctx *ctx, const rts_tune *shape);

/* Differentiable WCSPH substeps (every particle active, symplectic Euler)
 * and their adjoint, for gradient-based inverse problems:
 *   rho_i = m (W(0) + sum_j W_ij + sum_w W_iw),  p_i = B ((rho_i/rho0)^7 - 1)
 *   a_i = g - sum_j m (P_i + P_j + Pi_ij) gradW_ij - sum_w m (2 P_i + Pi_iw) gradW_iw
 *   v' = v + dt a,  x' = x + dt v'
 * with P = p / rho^2, Monaghan viscosity Pi_ij = -nu (v_ij . x_ij) /
 * (r^2 + eps h^2) for approaching pairs, nu = 2 alpha h c0 / (rho_i + rho_j)
 * (walls: at rest, mirrored density and pressure, nu = alpha h c0 / rho_i).
 * The pressure is not clamped.  The forward run keeps the state every
 * ckpt_every substeps in the caller's tape; the backward run recomputes each
 * segment from its checkpoint and runs the adjoint kernels in reverse.
 * These calls use the context's particle buffers as scratch: the context's
 * own simulation state is lost (set a state again before rts_advance). */
typedef struct rts_diff_desc {
  int32_t n_sub;          /* substeps */
  int32_t ckpt_every;     /* substeps between checkpoints */
  int32_t list_cap;       /* neighbour entries per particle (fluid + walls) */
  int32_t pad;
  double dt;              /* substep length */
  double B;               /* Tait stiffness (differentiated) */
  double alpha;           /* viscosity alpha (differentiated) */
} rts_diff_desc;

/* Device bytes of the tape for n particles. */
rts_status rts_diff_tape_bytes(rts_ctx *ctx, const rts_diff_desc *desc, int64_t n, size_t *bytes);
/* Runs the substeps from d_x0, d_v0 (planes, 3n floats) and writes the final
 * state to d_xT, d_vT (planes).  Asynchronous. */
rts_status rts_diff_forward(rts_ctx *ctx, const rts_diff_desc *desc, int64_t n, const float *d_x0,
                            const float *d_v0, float *d_xT, float *d_vT, void *d_tape,
                            size_t tape_bytes);
/* Given dL/dx(T) and dL/dv(T) (planes; d_vT_bar may be NULL for zero),
 * writes dL/dx(0), dL/dv(0) (planes; either may be NULL) and the host
 * values dL/dB, dL/dalpha.  Needs the tape of the forward run with the same
 * desc and n.  Waits for the stream. */
rts_status rts_diff_backward(rts_ctx *ctx, const rts_diff_desc *desc, int64_t n,
                             const float *d_xT_bar, const float *d_vT_bar, float *d_x0_bar,
                             float *d_v0_bar, double *h_B_bar, double *h_alpha_bar, void *d_tape,
                             size_t tape_bytes);

const char *rts_last_error(const rts_ctx *ctx);
const char *rts_status_string(rts_status s);

#ifdef __cplusplus
}
#endif
#endif /* RTS_H */
