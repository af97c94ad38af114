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
} orc_cfg;

typedef struct orc_info {
  int32_t nc[3];
  int64_t nblocks;
  float o[3];
  float inv_e, r2f;
  double mass, B, sigma, dt_base;
  float TV[ORC_MAX_LEVELS], TA[ORC_MAX_LEVELS];
  int32_t lmax;
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
void orc_flags(int32_t n, const uint32_t *key, const uint8_t *blk, int32_t *level,
               int32_t *validity, uint8_t *compute);
int  orc_neighbors(const orc_cfg *c, int32_t n, const float *pos, int32_t nw, const float *wpos,
                   const uint8_t *want, int32_t cap, uint32_t *nbr, int32_t *nnb);

/* physics, double precision */
int orc_density(const orc_cfg *c, int32_t n, const double *x, int32_t nw, const double *wx,
                const uint8_t *which, double *rho, double *p);
int orc_forces(const orc_cfg *c, int32_t n, const double *x, const double *v, const double *rho,
               const double *p, int32_t nw, const double *wx, const uint8_t *which, double *acc);

/* integrator pieces (Serna predictor-corrector) */
void orc_serna_predict(int32_t n, double *x, double *v, const double *a, double dt);
void orc_serna_correct(int32_t n, double *x, double *v, double *a, const double *a_new,
                       const double *dtau, const uint8_t *which);

/* one base step of Algorithm 1 (or of a global comparator) */
int orc_wcsph_step(const orc_cfg *c, orc_state *s);

int orc_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
