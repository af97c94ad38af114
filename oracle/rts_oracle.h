/*
 * rts_oracle.h -- plain CPU reference for regional time stepping (RTS) SPH.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no source
 * with the HIP library; the two meet only through the seeded scene arrays.
 *
 * Physics is double precision.  Decisions that turn floating point into an
 * integer (block keys, the neighbour predicate, block levels) are taken in
 * float, in the operation order fixed in the comments of rts_oracle.c, so
 * that they can be compared bit for bit with the single-precision GPU path.
 *
 * Array conventions: positions, velocities and accelerations are
 * array-of-structs, element 3*i + c.  Fluid neighbour ids are input indices;
 * wall neighbour ids carry bit 31 (0x80000000 | wall input index).
 */
#ifndef RTS_ORACLE_H
#define RTS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_E_INVALID = 1, ORC_E_CAPACITY = 2, ORC_E_NUMERICAL = 4 };
enum { ORC_MODE_RTS = 0, ORC_MODE_GLOBAL_FIXED = 1, ORC_MODE_GLOBAL_ADAPTIVE = 2 };
enum { ORC_WCSPH = 0, ORC_PCISPH = 1 };
#define ORC_MAX_LEVELS 8
#define ORC_WALL_BIT 0x80000000u
#define ORC_EMPTY_BLOCK 0xFFu

typedef struct orc_cfg {
  double spacing, h, support, block_edge;
  double rho0, mass;                 /* mass <= 0: calibrated on the rest lattice */
  double c0, gamma, B;               /* B <= 0: rho0 c0^2 / gamma */
  double visc_alpha, visc_eps;
  double g[3];
  double dom_min[3], dom_max[3];
  double dt_base;                    /* <= 0: lambda_v * r_crit / c0 */
  double r_crit;                     /* length r of Eq. 1-3; <= 0: support radius */
  double lambda_v, lambda_f, alpha_rts, beta2, beta_ratio;
  int32_t n_levels, level_cap, mode, clamp_p, serna_correct, nbr_cap;
  /* PCISPH (solver = ORC_PCISPH) */
  int32_t solver;
  int32_t n_minor;                   /* minor steps per major step (4) */
  int32_t it_min, it_max;            /* correction iterations: at least / at most (3, 50) */
  int32_t expand_layers;             /* dilation of regions 1 and 2, in blocks (4) */
  int32_t local_fail;                /* local iterations before reverting to global (3) */
  int32_t global_limit;              /* global iterations that end a major step early (6) */
  int32_t short_majors;              /* clean major steps before the long major returns (10) */
  int32_t two_ring_levels;           /* regions searching two block layers (<= 0: 1, region 1) */
  double eta, eta_T;                 /* max / average compression error thresholds */
  double delta;                      /* <= 0: from the prototype neighbourhood */
  double r_list;                     /* neighbour-list radius; <= 0: block edge */
  /* adaptive base step of regional PCISPH (orc_pci_next_dt) */
  int32_t adapt_dt;                  /* 1: adapt dt_base between major steps (RTS mode) */
  int32_t grow_iters;                /* grow after a major step none of whose minor steps
                                        needed more iterations (<= 0: it_min) */
  int32_t shrink_iters;              /* shrink after one where a minor step needed more
                                        (<= 0: it_min) */
  int32_t pad_adapt;
  double dt_min, dt_max;             /* bounds of the adapted step (<= 0: dt_base/4, 4 dt_base) */
  double grow, shrink;               /* factors after an easy / an overrun major step */
  /* WCSPH: 1 = a particle that takes level l is next due at the next base
   * step that is a multiple of 2^l (so every particle of a level updates on
   * the same steps); 0 = 2^l base steps after the current one (Algorithm 1
   * as printed) */
  int32_t phase_align;
  int32_t pad_phase;
} orc_cfg;

typedef struct orc_info {
  int32_t nc[3];
  int64_t nblocks;
  float o[3];
  float inv_e, r2f;
  double mass, B, sigma, dt_base;
  float TV[ORC_MAX_LEVELS], TA[ORC_MAX_LEVELS];
  int32_t lmax;
  float r2l;                         /* PCISPH list radius squared, in float */
  double delta;                      /* PCISPH pressure coefficient */
} orc_info;

typedef struct orc_state {
  int32_t n, nw;
  double *x, *v, *a, *rho, *p;       /* 3n, 3n, 3n, n, n */
  int32_t *level, *validity, *age;   /* n */
  uint8_t *compute;                  /* n */
  const double *wx;                  /* 3nw */
  double t, dt_prev;
  int64_t step;
  /* statistics of the last step */
  int32_t n_active;
  int64_t n_inter;
  double err_max;
  int32_t hist[ORC_MAX_LEVELS];
} orc_state;

int orc_derive(const orc_cfg *c, orc_info *out);

/* kernel and equation of state */
double orc_kernel_W(const orc_cfg *c, double r);
double orc_kernel_dWdr(const orc_cfg *c, double r);
double orc_lattice_sum(const orc_cfg *c);
double orc_eos(const orc_cfg *c, double rho);

/* structural steps, float decisions */
void orc_keys(const orc_cfg *c, int32_t n, const float *pos, uint32_t *key);
int  orc_sort(int64_t nb, int32_t n, const uint32_t *key, uint32_t *perm, uint32_t *cell_start);
void orc_block_levels(const orc_cfg *c, int32_t n, const uint32_t *key, const float *vel,
                      const float *acc, uint8_t *lvl);
void orc_rmin(const orc_cfg *c, const uint8_t *lvl_in, uint8_t *lvl_out);
/* W5 at base step `step` (the number of steps taken before it). */
void orc_flags(int32_t n, const uint32_t *key, const uint8_t *blk, int32_t *level,
               int32_t *validity, uint8_t *compute, int64_t step, int32_t phase_align);
int  orc_neighbors(const orc_cfg *c, int32_t n, const float *pos, int32_t nw, const float *wpos,
                   const uint8_t *want, int32_t cap, uint32_t *nbr, int32_t *nnb);

/* physics, double precision */
int orc_density(const orc_cfg *c, int32_t n, const double *x, int32_t nw, const double *wx,
                const uint8_t *which, double *rho, double *p);
int orc_forces(const orc_cfg *c, int32_t n, const double *x, const double *v, const double *rho,
               const double *p, int32_t nw, const double *wx, const uint8_t *which, double *acc);
/* The same, also giving per particle the sum of the magnitudes of the terms
 * that make up its acceleration, |g| + sum_j |m coef_ij gradW_ij|: the scale
 * against which a float evaluation's error is measured. */
int orc_forces_terms(const orc_cfg *c, int32_t n, const double *x, const double *v,
                     const double *rho, const double *p, int32_t nw, const double *wx,
                     const uint8_t *which, double *acc, double *tsum);

/* integrator pieces (Serna predictor-corrector) */
void orc_serna_predict(int32_t n, double *x, double *v, const double *a, double dt);
void orc_serna_correct(int32_t n, double *x, double *v, double *a, const double *a_new,
                       const double *dtau, const uint8_t *which);

/* one base step of Algorithm 1 (or of a global comparator) */
int orc_wcsph_step(const orc_cfg *c, orc_state *s);
/* step of the global adaptive comparator from the accelerations a (3n):
 * min(lambda_v r / c0, lambda_f sqrt(r / max|a|)) */
double orc_adaptive_dt(const orc_cfg *c, int32_t n, const double *a);

/* ---------------------------------------------------------------------- */
/* PCISPH with regional iteration counts (Section 5, Algorithms 2 and 3).   */
/* Block levels k = 0..3 stand for regions n = k + 1 (step n dt_b).         */
/* ---------------------------------------------------------------------- */
typedef struct orc_pci_state {
  int32_t n, nw;
  /* particle arrays, in the block order of the current major step */
  double *x, *v;                     /* 3n */
  double *fvg, *fp;                  /* 3n: non-pressure / pressure acceleration */
  double *p, *rho, *err;             /* n: pressure, predicted density, relative error */
  int32_t *region, *validity;        /* n */
  uint8_t *compute, *in_se;          /* n */
  uint32_t *id;                      /* n: caller index held in each slot */
  uint32_t *key;                     /* n: block of the major step's grid */
  uint32_t *nbr;                     /* n * nbr_cap: lists (sorted fluid index, walls | bit 31) */
  int32_t *nnb;                      /* n */
  /* blocks */
  uint32_t *cell_start;              /* nb + 1 */
  uint8_t *blk_level, *blk_ob;       /* nb: level (region - 1, 0xFF empty), observed flag */
  /* walls, static, in their own block order */
  const double *wx;                  /* 3nw (sorted by the caller-independent wall grid) */
  uint32_t *wcell_start;             /* nb + 1 */
  /* schedule and statistics */
  int32_t major_len, minor_in_major, clean_majors, major_excess;
  int64_t minor_steps;
  double t;
  int32_t last_iters, last_global_iters, last_resets, last_reverts, last_early_end;
  int32_t last_lists;                /* lists rebuilt in the last minor step */
  int64_t evals_density, evals_force; /* particle evaluations in the last minor step */
  double last_errmax, last_avg;
  int32_t hist[4];                   /* particles per region at the last minor step */
  /* adaptive base step */
  double dt_cur;                     /* step of the current major step (<= 0: cfg dt_base) */
  double last_dt;                    /* length of the last minor step */
  int32_t peak_iters;                /* most iterations of a minor step in this major step */
  int32_t pad_;
  float last_v2max, last_a2max;      /* speed^2 / acceleration^2 maxima at the last major end */
  /* roll-back of a major step whose correction failed to converge */
  double *snap;                      /* 15n: x, v, fvg, fp (3n each), p, rho, err */
  uint32_t *snap_id;                 /* n */
  double snap_t;
  int64_t snap_steps;
  int32_t snap_major_len, snap_clean;
  int32_t rollbacks;                 /* major steps rolled back so far */
  int32_t last_rollback;             /* 1: the last call rolled its major step back */
  /* optional record of the last minor step's correction iterations (for
   * tests); trace == NULL records nothing */
  struct orc_pci_iter_rec *trace;    /* trace_cap records */
  double *trace_p;                   /* NULL or trace_cap * n: p after each iteration */
  double *trace_e;                   /* NULL or trace_cap * n: relative density error of the
                                        particles evaluated in each iteration, NaN for the rest */
  int32_t trace_cap, trace_len;
} orc_pci_state;

/* Algorithm 3: the control of one minor step's correction loop.  The loop
 * runs while (iter <= min_iter or the maximum error >= eta) and
 * iter <= it_max.  After each iteration (C5-C6):
 *   global_iters counts the iterations that followed the schedule;
 *   iter and row advance;
 *   once the three scheduled rows are done (iter > 3) and the maximum error
 *   is still >= eta, min_iter grows by one and (regional mode only)
 *     - if the average error >= eta_T: the schedule restarts at row 1
 *       (global); a local phase that was running is abandoned and the
 *       pressure restored from the snapshot (a revert);
 *     - else, once the minor step's local phase has ended unconverged
 *       (local_off): the schedule restarts at row 1 (global);
 *     - else, if global: local iterations on S_e begin, with a snapshot of
 *       the pressure;
 *     - else, after local_fail local iterations without convergence: back to
 *       global at row 1 with the pressure restored (a revert).
 *   A minor step thus runs at most one local phase: local correction is
 *   chosen once, and the switch back to global corrections after it fails
 *   holds for the rest of the minor step.
 * Standard PCISPH (every region in every iteration) only grows min_iter. */
typedef struct orc_pci_ctl {
  int32_t iter;                      /* number of the next iteration, from 1 */
  int32_t row;                       /* schedule row of the next iteration, from 1 */
  int32_t min_iter;                  /* minIterations, from it_min */
  int32_t global;                    /* 1: next iteration follows the schedule */
  int32_t local_iters;               /* local iterations since the local phase began */
  int32_t global_iters;              /* iterations that followed the schedule */
  int32_t resets;                    /* schedule restarts */
  int32_t reverts;                   /* pressure restorations */
  int32_t local_off;                 /* 1 once the minor step's local phase ended */
} orc_pci_ctl;
enum { ORC_CTL_KEEP = 0, ORC_CTL_BACKUP = 1, ORC_CTL_RESTORE = 2 };

typedef struct orc_pci_iter_rec {
  int32_t iter;                      /* iteration number (1-based) */
  int32_t row;                       /* schedule row it used (global) */
  int32_t global;                    /* 1: it followed the schedule */
  uint32_t turn;                     /* regions with the turn (bit n-1: region n) */
  int32_t action;                    /* ORC_CTL_* taken after it */
  int32_t n_density, n_force;        /* particles evaluated */
  int32_t n_se;                      /* |S_e| after it */
  double errmax, avg;                /* errors after it */
} orc_pci_iter_rec;

void orc_pci_ctl_init(const orc_cfg *c, orc_pci_ctl *k);
/* 1 while another iteration is due (errmax: after the last iteration;
 * +infinity before the first) */
int orc_pci_ctl_more(const orc_cfg *c, const orc_pci_ctl *k, double errmax);
/* regions with the turn in the next iteration of minor-step column col */
uint32_t orc_pci_ctl_turn(const orc_pci_ctl *k, int32_t col, int32_t standard);
/* C5-C6 after an iteration with the given errors; returns ORC_CTL_BACKUP
 * (snapshot p) or ORC_CTL_RESTORE (p from the snapshot) or ORC_CTL_KEEP. */
int orc_pci_ctl_after(const orc_cfg *c, orc_pci_ctl *k, int32_t standard, double errmax,
                      double avg);
/* End of a minor step that took global_iters scheduled iterations (Section 5,
 * extra iterations): counts it in the major step; more than global_limit
 * global iterations mark the major step as overrun and end it early when
 * minor steps remain; at its end an overrun major step shortens the next
 * ones to 2 minor steps, and after short_majors clean major steps the length
 * returns to n_minor.  Returns 1 when the major step ends here.  Uses and
 * updates major_len, minor_in_major, clean_majors, major_excess,
 * last_early_end of s. */
int orc_pci_major_length(const orc_cfg *c, orc_pci_state *s, int32_t global_iters,
                         int32_t standard);
/* S7 (Section 5, neighbourhood updates): a particle whose speed or
 * acceleration (float, squared as for the regions) exceeds its region's
 * Eq. 2-3 bounds takes its block and the occupied blocks around it to the
 * largest region it satisfies; the particles of a block whose region fell
 * take that region, recompute their lists next minor step and restart
 * their validity; the observed blocks follow the new regions.  vel, acc:
 * 3n floats.  Returns 1 if a block changed. */
int orc_pci_smaller_steps(const orc_cfg *c, int32_t n, const uint32_t *key, const float *vel,
                          const float *acc, int32_t major_len, int32_t *region,
                          int32_t *validity, uint8_t *compute, uint8_t *blk_level,
                          uint8_t *blk_ob);
/* validity of a particle of region n: 1, 2, or the major-step length */
int32_t orc_pci_region_validity(int32_t region, int32_t major_len);

/* a19: delta = -1 / (beta (-sum gradW . sum gradW - sum gradW . gradW)),
 * beta = 2 (m dt_b / rho0)^2, over the full rest-lattice neighbourhood. */
double orc_pci_delta(const orc_cfg *c);
/* a13: block levels from Eq. 2-3 (alpha = 1, no Eq. 1), dilation of levels
 * 0 and 1 by expand_layers, R_min, observed blocks.  raw, lvl, ob: nb. */
void orc_pci_regions(const orc_cfg *c, int32_t n, const uint32_t *key, const float *vel,
                     const float *acc, uint8_t *raw, uint8_t *lvl, uint8_t *ob);
/* Dilation of one level by `layers` blocks (Chebyshev), occupied blocks only. */
void orc_pci_dilate(const orc_cfg *c, const uint8_t *in, uint8_t *out, int level, int layers);
/* Observed blocks: occupied, with an occupied 26-neighbour of smaller level. */
void orc_pci_observed(const orc_cfg *c, const uint8_t *lvl, uint8_t *ob);
/* a14: lists of the sorted particles with want[i] set, against the stored
 * grid: rings[i] block layers around block key[i], float predicate with the
 * list radius, canonical order (fluid sorted index ascending, then walls). */
int orc_pci_lists(const orc_cfg *c, int32_t n, const float *pos, const uint32_t *cell_start,
                  const uint32_t *key, int32_t nw, const float *wpos,
                  const uint32_t *wcell_start, const uint8_t *want, const uint8_t *rings,
                  int32_t cap, uint32_t *nbr, int32_t *nnb);
/* Density predicted at positions xs for particles with which[i] set (walls
 * at wx): rho = m (W(0) + sum_j W + sum_w W) over the stored lists. */
void orc_pci_density(const orc_cfg *c, int32_t n, const double *xs, const double *wx,
                     const uint32_t *nbr, const int32_t *nnb, const uint8_t *which,
                     double *rho);
/* Pressure acceleration -m sum_j (p_i/rho_i^2 + p_j/rho_j^2) gradW at xs;
 * a wall mirrors p_i and rho_i. */
void orc_pci_pressure_force(const orc_cfg *c, int32_t n, const double *xs, const double *wx,
                            const double *p, const double *rho, const uint32_t *nbr,
                            const int32_t *nnb, const uint8_t *which, double *fp);
/* The same with tsum[i] = sum_j |m (p_i/rho_i^2 + p_j/rho_j^2) gradW_ij|
 * (tsum may be NULL). */
void orc_pci_pressure_force_terms(const orc_cfg *c, int32_t n, const double *xs,
                                  const double *wx, const double *p, const double *rho,
                                  const uint32_t *nbr, const int32_t *nnb, const uint8_t *which,
                                  double *fp, double *tsum);
/* Gravity plus artificial viscosity (nu = alpha h c0 / rho0) at x, v. */
void orc_pci_nonpressure(const orc_cfg *c, int32_t n, const double *x, const double *v,
                         const double *wx, const uint32_t *nbr, const int32_t *nnb,
                         const uint8_t *which, double *fvg);
/* Schedule of Figure "iterations": regions (bit n-1 for region n) that take
 * row `row` (1..3) of minor-step column `col` (0..3).  The figure is not in
 * the text; the table meets every constraint the text states (pinned by a
 * test), but its equality with the paper's own table is parity unpinned. */
uint32_t orc_pci_turn(int32_t col, int32_t row);
/* One minor step of Algorithm 2 (a major step begins when due). */
int orc_pci_step(const orc_cfg *c, orc_pci_state *s);
/* With adapt_dt, a minor step whose correction still exceeds eta after
 * it_max iterations rolls its major step back to the state it started from
 * and restarts it with half the step (not below dt_min): the
 * call then leaves minor_steps and t as they were before the major step.
 * The paper only suggests adapting the base step; this rule is a reading,
 * pinned against its own stated properties, and its parity with the paper
 * is unpinned (there is no rule there to compare with).
 * Base step of the next major step (adapt_dt): dt scaled by shrink after a
 * major step that overran global_limit or had a minor step needing more than
 * shrink_iters iterations, else by grow after one whose minor steps all
 * needed at most grow_iters iterations, then capped by dt_max and by
 * Eq. 3 with beta_2 (alpha beta_2 r / V_max) and Eq. 2 (lambda_f
 * sqrt(r / A_max)) of the fastest particle, and raised to dt_min.
 * v2max, a2max: squared maxima, in float. */
double orc_pci_next_dt(const orc_cfg *c, double dt, int32_t peak_iters, int32_t excess,
                       float v2max, float a2max);
/* Major-step set-up alone: sort into the grid, regions, flags. */
int orc_pci_major_begin(const orc_cfg *c, orc_pci_state *s);

/* ---------------------------------------------------------------------- */
/* Differentiable WCSPH substep (every particle active, symplectic Euler):  */
/*   rho_i = m (W(0) + sum_j W_ij + sum_w W_iw)                             */
/*   p_i   = B ((rho_i / rho0)^7 - 1)            (no clamp)                 */
/*   a_i   = g - sum_j m (P_i + P_j + Pi_ij) gradW_ij                       */
/*             - sum_w m (2 P_i + Pi_iw) gradW_iw,   P = p / rho^2           */
/*   Pi_ij = -nu_ij (v_ij . x_ij) / (r^2 + eps h^2) if v_ij . x_ij < 0,      */
/*   nu_ij = 2 alpha h c0 / (rho_i + rho_j), nu_iw = alpha h c0 / rho_i      */
/*   v' = v + dt a ;  x' = x + dt v'                                         */
/* and its adjoint for L = mean_i |x_i(T) - xhat_i|^2.                      */
/* ---------------------------------------------------------------------- */
int orc_diff_run(const orc_cfg *c, int32_t n, const double *x0, const double *v0, int32_t nw,
                 const double *wx, double B, double alpha, double dt, int32_t n_sub,
                 double *x_out, double *v_out);
int orc_diff_grad(const orc_cfg *c, int32_t n, const double *x0, const double *v0, int32_t nw,
                  const double *wx, double B, double alpha, double dt, int32_t n_sub,
                  const double *xhat, double *loss, double *g_x0, double *g_v0, double *g_B,
                  double *g_alpha);

int orc_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
