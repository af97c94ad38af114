/*
 * rts_oracle.c -- plain CPU reference for regional time stepping SPH.
 *
 * TEST INFRASTRUCTURE ONLY (see rts_oracle.h).  Written for clarity, not
 * speed: every step follows the paper's order and notation.
 *
 * Paper: Goswami & Batty, "Asynchronous Liquids: Regional Time Stepping for
 * Faster SPH and PCISPH".  Section references below are to that paper.
 *
 * Compile with -ffp-contract=off: the float decisions below must not be
 * fused into FMAs.
 */
#include "rts_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Kernel: the M4 cubic spline with support 2h (Monaghan 2005).  The paper    */
/* delegates the SPH discretisation to the cited WCSPH works; the scene fixes */
/* "cubic spline, h = 2 x spacing".  sigma = 1 / (pi h^3), q = |x| / h.        */
/* ------------------------------------------------------------------------ */
static double w_shape(double q) {
  if (q < 1.0) return 1.0 - 1.5 * q * q + 0.75 * q * q * q;
  if (q < 2.0) { double t = 2.0 - q; return 0.25 * t * t * t; }
  return 0.0;
}
static double dw_shape(double q) { /* d w_shape / dq */
  if (q < 1.0) return -3.0 * q + 2.25 * q * q;
  if (q < 2.0) { double t = 2.0 - q; return -0.75 * t * t; }
  return 0.0;
}
double orc_kernel_W(const orc_cfg *c, double r) {
  double sigma = 1.0 / (M_PI * c->h * c->h * c->h);
  return sigma * w_shape(r / c->h);
}
double orc_kernel_dWdr(const orc_cfg *c, double r) {
  double sigma = 1.0 / (M_PI * c->h * c->h * c->h);
  return sigma * dw_shape(r / c->h) / c->h;
}

/* Sum of W over an infinite cubic lattice of spacing s around one site
 * (self included).  Particle mass is rho0 / this sum, so that a particle in
 * the interior of the rest lattice has exactly the rest density. */
double orc_lattice_sum(const orc_cfg *c) {
  double s = c->spacing, r = c->support;
  int m = (int)ceil(r / s) + 1;
  double sum = 0.0;
  for (int k = -m; k <= m; ++k)
    for (int j = -m; j <= m; ++j)
      for (int i = -m; i <= m; ++i) {
        double d = s * sqrt((double)(i * i + j * j + k * k));
        if (d < r) sum += orc_kernel_W(c, d);
      }
  return sum;
}

static double tait_B(const orc_cfg *c) {
  return c->B > 0.0 ? c->B : c->rho0 * c->c0 * c->c0 / c->gamma;
}

/* Tait equation of state p = B ((rho / rho0)^gamma - 1) (Becker & Teschner),
 * clamped at zero when clamp_p is set. */
double orc_eos(const orc_cfg *c, double rho) {
  double p = tait_B(c) * (pow(rho / c->rho0, c->gamma) - 1.0);
  if (c->clamp_p && p < 0.0) p = 0.0;
  return p;
}

static double r_crit(const orc_cfg *c) { return c->r_crit > 0.0 ? c->r_crit : c->support; }

static double base_dt(const orc_cfg *c) {
  /* Eq. 1 with the base step at its bound when no step is given. */
  return c->dt_base > 0.0 ? c->dt_base : c->lambda_v * r_crit(c) / c->c0;
}

static double beta_n(const orc_cfg *c, int n) {
  /* Section 3.1: beta_1 = infinity, beta_n = 0.4 * 0.2^(n-2) for n >= 2. */
  if (n <= 1) return INFINITY;
  return c->beta2 * pow(c->beta_ratio, (double)(n - 2));
}

int orc_derive(const orc_cfg *c, orc_info *o) {
  memset(o, 0, sizeof(*o));
  if (!(c->spacing > 0 && c->h > 0 && c->support > 0 && c->block_edge >= c->support &&
        c->rho0 > 0 && c->c0 > 0 && c->n_levels >= 1 && c->n_levels <= ORC_MAX_LEVELS))
    return ORC_E_INVALID;
  int64_t nb = 1;
  for (int d = 0; d < 3; ++d) {
    double ext = c->dom_max[d] - c->dom_min[d];
    if (!(ext > 0)) return ORC_E_INVALID;
    o->nc[d] = (int32_t)ceil(ext / c->block_edge);
    if (o->nc[d] < 1) o->nc[d] = 1;
    nb *= o->nc[d];
    o->o[d] = (float)c->dom_min[d];
  }
  o->nblocks = nb;
  o->inv_e = (float)(1.0 / c->block_edge);
  o->r2f = (float)(c->support * c->support);
  o->sigma = 1.0 / (M_PI * c->h * c->h * c->h);
  o->mass = c->mass > 0.0 ? c->mass : c->rho0 / orc_lattice_sum(c);
  o->B = tait_B(c);
  o->dt_base = base_dt(c);
  int lmax = c->n_levels - 1;
  if (c->level_cap < lmax) lmax = c->level_cap < 0 ? 0 : c->level_cap;
  if (c->mode != ORC_MODE_RTS) lmax = 0;
  o->lmax = lmax;
  /* WCSPH level l steps 2^l base steps; PCISPH level l is region n = l + 1,
   * stepping n base steps (Section 5).  Either way l is ranked n = l + 1
   * for beta (Eq. 3):
   *   Eq. 3:  dt_l |v| / r <= alpha beta_{l+1}  ->  |v|^2 <= TV[l]
   *   Eq. 2:  dt_l <= lambda_f sqrt(r / |a|)    ->  |a|^2 <= TA[l]   */
  for (int l = 0; l < ORC_MAX_LEVELS; ++l) {
    double dtl = c->solver == ORC_PCISPH ? o->dt_base * (double)(l + 1) : ldexp(o->dt_base, l);
    double b = beta_n(c, l + 1);
    double vl = isinf(b) ? INFINITY : c->alpha_rts * b * r_crit(c) / dtl;
    double al = c->lambda_f * c->lambda_f * r_crit(c) / (dtl * dtl);
    o->TV[l] = (float)(vl * vl);
    o->TA[l] = (float)(al * al);
  }
  if (c->solver == ORC_PCISPH) {
    double rl = c->r_list > 0.0 ? c->r_list : c->block_edge;
    o->r2l = (float)(rl * rl);
    o->delta = c->delta > 0.0 ? c->delta : orc_pci_delta(c);
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Block grid (Section 3).  Blocks have edge e >= support radius r, so all    */
/* neighbours of a particle lie in its own block or the 26 around it.         */
/* Key, in float:  t = x - o ; u = t * inv_e ; b = floor(u) clamped to        */
/* [0, n-1] ; key = bx + nx (by + ny bz).                                      */
/* ------------------------------------------------------------------------ */
static void block_coords(const orc_info *I, const float *p, int32_t b[3]) {
  for (int d = 0; d < 3; ++d) {
    float t = p[d] - I->o[d];
    float u = t * I->inv_e;
    float f = floorf(u);
    int32_t k;
    if (!(f >= 0.0f)) k = 0;           /* also catches NaN */
    else if (f >= (float)(I->nc[d] - 1)) k = I->nc[d] - 1;
    else k = (int32_t)f;
    b[d] = k;
  }
}
static uint32_t key_of(const orc_info *I, const int32_t b[3]) {
  return (uint32_t)(b[0] + I->nc[0] * (b[1] + I->nc[1] * b[2]));
}

void orc_keys(const orc_cfg *c, int32_t n, const float *pos, uint32_t *key) {
  orc_info I;
  orc_derive(c, &I);
  for (int32_t i = 0; i < n; ++i) {
    int32_t b[3];
    block_coords(&I, pos + 3 * (int64_t)i, b);
    key[i] = key_of(&I, b);
  }
}

/* Stable counting sort: perm[new] = old, ties kept in input order. */
int orc_sort(int64_t nb, int32_t n, const uint32_t *key, uint32_t *perm, uint32_t *cell_start) {
  memset(cell_start, 0, sizeof(uint32_t) * (size_t)(nb + 1));
  for (int32_t i = 0; i < n; ++i) {
    if ((int64_t)key[i] >= nb) return ORC_E_INVALID;
    cell_start[key[i] + 1]++;
  }
  for (int64_t b = 0; b < nb; ++b) cell_start[b + 1] += cell_start[b];
  uint32_t *fill = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(nb > 0 ? nb : 1));
  memcpy(fill, cell_start, sizeof(uint32_t) * (size_t)nb);
  for (int32_t i = 0; i < n; ++i) perm[fill[key[i]]++] = (uint32_t)i;
  free(fill);
  return ORC_OK;
}

/* |v|^2 in float, fixed order: (vx*vx + vy*vy) + vz*vz. */
static float norm2f(const float *v) {
  float xx = v[0] * v[0];
  float yy = v[1] * v[1];
  float zz = v[2] * v[2];
  float s = xx + yy;
  return s + zz;
}

/* Section 3.1 steps 1-2: each block takes the maxima of its particles'
 * speed and acceleration, then the largest level whose step satisfies Eq. 2
 * and Eq. 3 (Eq. 1 fixes the base step).  Empty blocks get 0xFF. */
void orc_block_levels(const orc_cfg *c, int32_t n, const uint32_t *key, const float *vel,
                      const float *acc, uint8_t *lvl) {
  orc_info I;
  orc_derive(c, &I);
  float *vm = (float *)calloc((size_t)I.nblocks, sizeof(float));
  float *am = (float *)calloc((size_t)I.nblocks, sizeof(float));
  uint8_t *occ = (uint8_t *)calloc((size_t)I.nblocks, 1);
  for (int32_t i = 0; i < n; ++i) {
    uint32_t b = key[i];
    float v2 = norm2f(vel + 3 * (int64_t)i), a2 = norm2f(acc + 3 * (int64_t)i);
    if (!occ[b] || v2 > vm[b]) vm[b] = v2;
    if (!occ[b] || a2 > am[b]) am[b] = a2;
    occ[b] = 1;
  }
  for (int64_t b = 0; b < I.nblocks; ++b) {
    if (!occ[b]) { lvl[b] = ORC_EMPTY_BLOCK; continue; }
    int l = 0;
    while (l + 1 <= I.lmax && vm[b] <= I.TV[l + 1] && am[b] <= I.TA[l + 1]) ++l;
    lvl[b] = (uint8_t)l;
  }
  free(vm); free(am); free(occ);
}

/* R_min (Section 4.2): a block next to a region of smaller step takes that
 * smaller step.  One pass over the 26 neighbours, occupied blocks only. */
void orc_rmin(const orc_cfg *c, const uint8_t *in, uint8_t *out) {
  orc_info I;
  orc_derive(c, &I);
  for (int32_t z = 0; z < I.nc[2]; ++z)
    for (int32_t y = 0; y < I.nc[1]; ++y)
      for (int32_t x = 0; x < I.nc[0]; ++x) {
        int32_t b[3] = {x, y, z};
        uint32_t k = key_of(&I, b);
        uint8_t l = in[k];
        if (l != ORC_EMPTY_BLOCK) {
          for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
              for (int dx = -1; dx <= 1; ++dx) {
                int32_t q[3] = {x + dx, y + dy, z + dz};
                if (q[0] < 0 || q[1] < 0 || q[2] < 0 || q[0] >= I.nc[0] || q[1] >= I.nc[1] ||
                    q[2] >= I.nc[2])
                  continue;
                uint8_t m = in[key_of(&I, q)];
                if (m < l) l = m;   /* 0xFF (empty) never wins */
              }
        }
        out[k] = l;
      }
}

/* Algorithm 1, particle flags: decrement validity; a particle is active when
 * its validity has run out or its block's step differs from its own (the
 * pre-emption rule); an active particle takes the block's step and a
 * validity of 2^level base steps. */
void orc_flags(int32_t n, const uint32_t *key, const uint8_t *blk, int32_t *level,
               int32_t *validity, uint8_t *compute, int64_t step, int32_t phase_align) {
  for (int32_t i = 0; i < n; ++i) {
    int32_t bl = blk[key[i]];
    validity[i] -= 1;
    if (validity[i] <= 0 || level[i] != bl) {
      /* due: the step of its block, for 2^l base steps (Algorithm 1), or
       * up to the next multiple of 2^l (phase-aligned) */
      const int32_t len = 1 << bl;
      compute[i] = 1;
      level[i] = bl;
      validity[i] = phase_align ? len - (int32_t)(step % len) : len;
    } else {
      compute[i] = 0;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Neighbour search over the block grid.  Predicate in float, fused:         */
/*   dx = xj - xi (per axis) ; d2 = fma(dz, dz, fma(dy, dy, dx*dx)) < r2f.   */
/* Canonical list order: fluid by sorted position ascending (blocks scanned  */
/* dz, dy, dx ascending), then walls by their sorted position ascending.     */
/* ------------------------------------------------------------------------ */
typedef struct {
  int64_t nb;
  uint32_t *key, *perm, *start;  /* perm: sorted position -> input index */
} grid_t;

static int grid_build(const orc_info *I, int32_t n, const float *pos, grid_t *g) {
  g->nb = I->nblocks;
  g->key = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
  g->perm = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
  g->start = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(g->nb + 1));
  for (int32_t i = 0; i < n; ++i) {
    int32_t b[3];
    block_coords(I, pos + 3 * (int64_t)i, b);
    g->key[i] = key_of(I, b);
  }
  return orc_sort(g->nb, n, g->key, g->perm, g->start);
}
static void grid_free(grid_t *g) { free(g->key); free(g->perm); free(g->start); }

static int near_f(const float *pi, const float *pj, float r2f) {
  float dx = pj[0] - pi[0];
  float dy = pj[1] - pi[1];
  float dz = pj[2] - pi[2];
  float xx = dx * dx;
  float d2 = fmaf(dz, dz, fmaf(dy, dy, xx));   /* fmaf rounds once per fused step */
  return d2 < r2f;
}

/* Neighbours of particle i (input index), appended in canonical order.
 * Returns the count, or -1 on overflow of cap. */
static int32_t find_neighbors(const orc_info *I, int32_t i, const float *pos, const grid_t *gf,
                              const float *wpos, const grid_t *gw, int32_t cap, uint32_t *out) {
  int32_t b[3], cnt = 0;
  const float *pi = pos + 3 * (int64_t)i;
  block_coords(I, pi, b);
  for (int pass = 0; pass < 2; ++pass) {
    const grid_t *g = pass == 0 ? gf : gw;
    const float *P = pass == 0 ? pos : wpos;
    if (!g) continue;
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          int32_t q[3] = {b[0] + dx, b[1] + dy, b[2] + dz};
          if (q[0] < 0 || q[1] < 0 || q[2] < 0 || q[0] >= I->nc[0] || q[1] >= I->nc[1] ||
              q[2] >= I->nc[2])
            continue;
          uint32_t k = key_of(I, q);
          for (uint32_t s = g->start[k]; s < g->start[k + 1]; ++s) {
            uint32_t j = g->perm[s];
            if (pass == 0 && (int32_t)j == i) continue;
            if (!near_f(pi, P + 3 * (int64_t)j, I->r2f)) continue;
            if (cnt >= cap) return -1;
            out[cnt++] = pass == 0 ? j : (ORC_WALL_BIT | j);
          }
        }
  }
  return cnt;
}

int orc_neighbors(const orc_cfg *c, int32_t n, const float *pos, int32_t nw, const float *wpos,
                  const uint8_t *want, int32_t cap, uint32_t *nbr, int32_t *nnb) {
  orc_info I;
  if (orc_derive(c, &I)) return ORC_E_INVALID;
  grid_t gf, gw;
  grid_build(&I, n, pos, &gf);
  grid_build(&I, nw, wpos, &gw);
  int status = ORC_OK;
#pragma omp parallel for schedule(dynamic, 64)
  for (int32_t i = 0; i < n; ++i) {
    if (want && !want[i]) { nnb[i] = 0; continue; }
    int32_t k = find_neighbors(&I, i, pos, &gf, wpos, nw > 0 ? &gw : NULL, cap,
                               nbr + (int64_t)i * cap);
    if (k < 0) {
#pragma omp atomic write
      status = ORC_E_CAPACITY;
      k = cap;
    }
    nnb[i] = k;
  }
  grid_free(&gf);
  grid_free(&gw);
  return status;
}

/* ------------------------------------------------------------------------ */
/* Physics in double precision.                                               */
/* ------------------------------------------------------------------------ */
typedef struct {
  orc_info I;
  int32_t n, nw, cap;
  float *pf, *wf;      /* float copies of positions for the predicate */
  grid_t gf, gw;
  uint32_t *nbr;
  int32_t *nnb;
} ctx_t;

static int ctx_open(ctx_t *X, const orc_cfg *c, int32_t n, const double *x, int32_t nw,
                    const double *wx) {
  memset(X, 0, sizeof(*X));
  if (orc_derive(c, &X->I)) return ORC_E_INVALID;
  X->n = n; X->nw = nw;
  X->cap = c->nbr_cap > 0 ? c->nbr_cap : 512;
  X->pf = (float *)malloc(sizeof(float) * 3 * (size_t)(n > 0 ? n : 1));
  X->wf = (float *)malloc(sizeof(float) * 3 * (size_t)(nw > 0 ? nw : 1));
  for (int64_t k = 0; k < 3 * (int64_t)n; ++k) X->pf[k] = (float)x[k];
  for (int64_t k = 0; k < 3 * (int64_t)nw; ++k) X->wf[k] = (float)wx[k];
  grid_build(&X->I, n, X->pf, &X->gf);
  grid_build(&X->I, nw, X->wf, &X->gw);
  X->nbr = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)X->cap * (size_t)(n > 0 ? n : 1));
  X->nnb = (int32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
  return ORC_OK;
}
static void ctx_close(ctx_t *X) {
  free(X->pf); free(X->wf); free(X->nbr); free(X->nnb);
  grid_free(&X->gf); grid_free(&X->gw);
}
static int ctx_lists(ctx_t *X, const uint8_t *which) {
  int status = ORC_OK;
#pragma omp parallel for schedule(dynamic, 64)
  for (int32_t i = 0; i < X->n; ++i) {
    if (which && !which[i]) { X->nnb[i] = 0; continue; }
    int32_t k = find_neighbors(&X->I, i, X->pf, &X->gf, X->wf, X->nw > 0 ? &X->gw : NULL,
                               X->cap, X->nbr + (int64_t)i * X->cap);
    if (k < 0) {
#pragma omp atomic write
      status = ORC_E_CAPACITY;
      k = 0;
    }
    X->nnb[i] = k;
  }
  return status;
}

/* Density by summation over the neighbourhood, self and walls included:
 * rho_i = m (W(0) + sum_j W(|x_i - x_j|)); then the Tait pressure. */
static void density_from_lists(const orc_cfg *c, ctx_t *X, const double *x, const double *wx,
                               const uint8_t *which, double *rho, double *p) {
  double m = X->I.mass;
#pragma omp parallel for schedule(dynamic, 64)
  for (int32_t i = 0; i < X->n; ++i) {
    if (which && !which[i]) continue;
    const double *xi = x + 3 * (int64_t)i;
    double sum = orc_kernel_W(c, 0.0);
    const uint32_t *L = X->nbr + (int64_t)i * X->cap;
    for (int32_t k = 0; k < X->nnb[i]; ++k) {
      uint32_t j = L[k];
      const double *xj = (j & ORC_WALL_BIT) ? wx + 3 * (int64_t)(j & ~ORC_WALL_BIT)
                                            : x + 3 * (int64_t)j;
      double d0 = xi[0] - xj[0], d1 = xi[1] - xj[1], d2 = xi[2] - xj[2];
      sum += orc_kernel_W(c, sqrt(d0 * d0 + d1 * d1 + d2 * d2));
    }
    rho[i] = m * sum;
    p[i] = orc_eos(c, rho[i]);
  }
}

/* Acceleration of particle i (Becker & Teschner WCSPH, Monaghan viscosity):
 *   a_i = g - sum_j m (p_i/rho_i^2 + p_j/rho_j^2) gradW_ij - sum_j m Pi_ij gradW_ij
 *   Pi_ij = -nu (v_ij . x_ij) / (|x_ij|^2 + eps h^2)  when v_ij . x_ij < 0
 *   nu = 2 alpha h c0 / (rho_i + rho_j)
 * Wall particles mirror the fluid particle's pressure and density and are
 * at rest. */
static void forces_from_lists(const orc_cfg *c, ctx_t *X, const double *x, const double *v,
                              const double *rho, const double *p, const double *wx,
                              const uint8_t *which, double *acc, double *tsum) {
  double m = X->I.mass, h = c->h;
#pragma omp parallel for schedule(dynamic, 64)
  for (int32_t i = 0; i < X->n; ++i) {
    if (which && !which[i]) continue;
    const double *xi = x + 3 * (int64_t)i, *vi = v + 3 * (int64_t)i;
    double ri = rho[i], pi = p[i];
    double ai[3] = {c->g[0], c->g[1], c->g[2]};
    double ts = sqrt(c->g[0] * c->g[0] + c->g[1] * c->g[1] + c->g[2] * c->g[2]);
    const uint32_t *L = X->nbr + (int64_t)i * X->cap;
    for (int32_t k = 0; k < X->nnb[i]; ++k) {
      uint32_t j = L[k];
      const double *xj;
      double vj[3], rj, pj;
      if (j & ORC_WALL_BIT) {
        xj = wx + 3 * (int64_t)(j & ~ORC_WALL_BIT);
        vj[0] = vj[1] = vj[2] = 0.0;
        rj = ri;
        pj = pi + ri * (c->g[0] * (xj[0] - xi[0]) + c->g[1] * (xj[1] - xi[1]) +
                        c->g[2] * (xj[2] - xi[2]));
        if (pj < 0.0) pj = 0.0;
      } else {
        xj = x + 3 * (int64_t)j;
        for (int d = 0; d < 3; ++d) vj[d] = v[3 * (int64_t)j + d];
        rj = rho[j]; pj = p[j];
      }
      double xij[3] = {xi[0] - xj[0], xi[1] - xj[1], xi[2] - xj[2]};
      double r2 = xij[0] * xij[0] + xij[1] * xij[1] + xij[2] * xij[2];
      double r = sqrt(r2);
      if (r == 0.0) continue;                       /* gradW(0) = 0 */
      double dw = orc_kernel_dWdr(c, r) / r;        /* gradW = dw * xij */
      double coef = pi / (ri * ri) + pj / (rj * rj);
      double vij[3] = {vi[0] - vj[0], vi[1] - vj[1], vi[2] - vj[2]};
      double vx = vij[0] * xij[0] + vij[1] * xij[1] + vij[2] * xij[2];
      if (vx < 0.0) {
        double nu = 2.0 * c->visc_alpha * h * c->c0 / (ri + rj);
        coef += -nu * vx / (r2 + c->visc_eps * h * h);
      }
      for (int d = 0; d < 3; ++d) ai[d] -= m * coef * dw * xij[d];
      ts += fabs(m * coef * dw) * r;
    }
    for (int d = 0; d < 3; ++d) acc[3 * (int64_t)i + d] = ai[d];
    if (tsum) tsum[i] = ts;
  }
}

int orc_density(const orc_cfg *c, int32_t n, const double *x, int32_t nw, const double *wx,
                const uint8_t *which, double *rho, double *p) {
  ctx_t X;
  if (ctx_open(&X, c, n, x, nw, wx)) return ORC_E_INVALID;
  int st = ctx_lists(&X, which);
  density_from_lists(c, &X, x, wx, which, rho, p);
  ctx_close(&X);
  return st;
}

int orc_forces(const orc_cfg *c, int32_t n, const double *x, const double *v, const double *rho,
               const double *p, int32_t nw, const double *wx, const uint8_t *which, double *acc) {
  ctx_t X;
  if (ctx_open(&X, c, n, x, nw, wx)) return ORC_E_INVALID;
  int st = ctx_lists(&X, which);
  forces_from_lists(c, &X, x, v, rho, p, wx, which, acc, NULL);
  ctx_close(&X);
  return st;
}

int orc_forces_terms(const orc_cfg *c, int32_t n, const double *x, const double *v,
                     const double *rho, const double *p, int32_t nw, const double *wx,
                     const uint8_t *which, double *acc, double *tsum) {
  ctx_t X;
  if (ctx_open(&X, c, n, x, nw, wx)) return ORC_E_INVALID;
  int st = ctx_lists(&X, which);
  forces_from_lists(c, &X, x, v, rho, p, wx, which, acc, tsum);
  ctx_close(&X);
  return st;
}

/* ------------------------------------------------------------------------ */
/* Serna predictor-corrector (Section 4.1).                                   */
/*   predictor, all particles:  x~ = x + v dt + a dt^2 / 2 ;  v~ = v + a dt   */
/*   corrector, active only:    x = x~ + (a_new - a) dtau^2 / 6               */
/*                              v = v~ + (a_new - a) dtau / 2                 */
/* dtau is the time since the particle's last acceleration evaluation.        */
/* ------------------------------------------------------------------------ */
void orc_serna_predict(int32_t n, double *x, double *v, const double *a, double dt) {
  for (int64_t k = 0; k < 3 * (int64_t)n; ++k) {
    x[k] += v[k] * dt + 0.5 * a[k] * dt * dt;
    v[k] += a[k] * dt;
  }
}

void orc_serna_correct(int32_t n, double *x, double *v, double *a, const double *a_new,
                       const double *dtau, const uint8_t *which) {
  for (int32_t i = 0; i < n; ++i) {
    if (which && !which[i]) continue;
    double t = dtau[i];
    for (int d = 0; d < 3; ++d) {
      int64_t k = 3 * (int64_t)i + d;
      double da = a_new[k] - a[k];
      x[k] += da * t * t / 6.0;
      v[k] += da * t / 2.0;
      a[k] = a_new[k];
    }
  }
}

/* ------------------------------------------------------------------------ */
/* One base step of Algorithm 1.  Order within the step:                      */
/*   W1 block grid on the predicted positions                                 */
/*   W2 block maxima of |v|^2, |a|^2 (stored acceleration, gravity included)  */
/*   W3 block level from Eq. 2 and Eq. 3                                      */
/*   W4 R_min                                                                 */
/*   W5 particle flags (validity, compute, pre-emption)                       */
/*   W6-W8 neighbours, density + pressure, acceleration for active particles; */
/*         inactive neighbours contribute their last density and pressure     */
/*   W9 corrector for active particles                                        */
/*   W10 predictor for all particles                                          */
/* The corrector of the step that ends now precedes the predictor of the next */
/* one, as the predictor-corrector equations require.  The global comparators */
/* are the same loop with every block at level 0; the adaptive one takes     */
/* dt = min(lambda_v r / c0, lambda_f sqrt(r / max|a|)) each step.            */
/* ------------------------------------------------------------------------ */
/* Global adaptive comparator: Eq. 1 and Eq. 2 for every particle at once,
 * dt = min(lambda_v r / c0, lambda_f sqrt(r / max|a|)). */
double orc_adaptive_dt(const orc_cfg *c, int32_t n, const double *a) {
  double amax2 = 0.0;
  for (int32_t i = 0; i < n; ++i) {
    const double *ai = a + 3 * (int64_t)i;
    double a2 = ai[0] * ai[0] + ai[1] * ai[1] + ai[2] * ai[2];
    if (a2 > amax2) amax2 = a2;
  }
  double dt = c->lambda_v * r_crit(c) / c->c0;
  if (amax2 > 0.0) {
    double df = c->lambda_f * sqrt(r_crit(c) / sqrt(amax2));
    if (df < dt) dt = df;
  }
  return dt;
}

int orc_wcsph_step(const orc_cfg *c, orc_state *s) {
  int32_t n = s->n;
  ctx_t X;
  if (ctx_open(&X, c, n, s->x, s->nw, s->wx)) return ORC_E_INVALID;
  const orc_info *I = &X.I;
  int status = ORC_OK;

  for (int32_t i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) {
      double q = s->x[3 * (int64_t)i + d];
      if (!isfinite(q) || !isfinite(s->v[3 * (int64_t)i + d]) || q < c->dom_min[d] ||
          q > c->dom_max[d])
        status = ORC_E_NUMERICAL;
    }
  if (status) { ctx_close(&X); return status; }

  /* W2-W4 */
  float *vf = (float *)malloc(sizeof(float) * 3 * (size_t)(n > 0 ? n : 1));
  float *af = (float *)malloc(sizeof(float) * 3 * (size_t)(n > 0 ? n : 1));
  for (int64_t k = 0; k < 3 * (int64_t)n; ++k) { vf[k] = (float)s->v[k]; af[k] = (float)s->a[k]; }
  uint8_t *lraw = (uint8_t *)malloc((size_t)I->nblocks);
  uint8_t *lvl = (uint8_t *)malloc((size_t)I->nblocks);
  orc_block_levels(c, n, X.gf.key, vf, af, lraw);
  orc_rmin(c, lraw, lvl);

  /* W5 */
  orc_flags(n, X.gf.key, lvl, s->level, s->validity, s->compute, s->step, c->phase_align);

  /* W6-W8 */
  status = ctx_lists(&X, s->compute);
  density_from_lists(c, &X, s->x, s->wx, s->compute, s->rho, s->p);
  double *anew = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
  forces_from_lists(c, &X, s->x, s->v, s->rho, s->p, s->wx, s->compute, anew, NULL);

  /* statistics */
  s->n_active = 0; s->n_inter = 0; s->err_max = 0.0;
  memset(s->hist, 0, sizeof(s->hist));
  for (int32_t i = 0; i < n; ++i) {
    if (s->compute[i]) { s->n_active++; s->n_inter += X.nnb[i]; }
    double e = (s->rho[i] - c->rho0) / c->rho0;
    if (e > s->err_max) s->err_max = e;
    if (s->level[i] >= 0 && s->level[i] < ORC_MAX_LEVELS) s->hist[s->level[i]]++;
  }

  /* W9: corrector; dtau = age * dt_base (RTS, fixed) or the last step (adaptive) */
  double *dtau = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  for (int32_t i = 0; i < n; ++i)
    dtau[i] = c->mode == ORC_MODE_GLOBAL_ADAPTIVE ? s->dt_prev : s->age[i] * I->dt_base;
  if (c->serna_correct) {
    orc_serna_correct(n, s->x, s->v, s->a, anew, dtau, s->compute);
  } else {
    for (int32_t i = 0; i < n; ++i)
      if (s->compute[i])
        for (int d = 0; d < 3; ++d) s->a[3 * (int64_t)i + d] = anew[3 * (int64_t)i + d];
  }
  for (int32_t i = 0; i < n; ++i)
    if (s->compute[i]) s->age[i] = 0;

  /* W10: predictor with this step's length */
  double dt = c->mode == ORC_MODE_GLOBAL_ADAPTIVE ? orc_adaptive_dt(c, n, s->a) : I->dt_base;
  orc_serna_predict(n, s->x, s->v, s->a, dt);
  for (int32_t i = 0; i < n; ++i) s->age[i] += 1;
  s->dt_prev = dt;
  s->t += dt;
  s->step += 1;

  free(vf); free(af); free(lraw); free(lvl); free(anew); free(dtau);
  ctx_close(&X);
  return status;
}

/* ======================================================================== */
/* PCISPH with regional iteration counts (Section 5, Algorithms 2 and 3).    */
/* Regions R_n, n = 1..4, are block levels l = n - 1; a region-n block is     */
/* corrected according to the schedule and its particles' neighbourhoods are */
/* refreshed every n minor steps (n <= 2) or once per major step (n >= 3).   */
/* ======================================================================== */

/* gradient of W at x_ij = x_i - x_j, |x_ij| = d > 0 */
static void grad_w(const orc_cfg *c, const double *xij, double d, double *g) {
  double f = d > 0.0 ? orc_kernel_dWdr(c, d) / d : 0.0;
  g[0] = f * xij[0]; g[1] = f * xij[1]; g[2] = f * xij[2];
}

/* a19.  The PCISPH pressure coefficient of Solenthaler & Pajarola (the
 * standard PCISPH the paper builds on): delta = -1 / (beta (-S.S - Q)) with
 * S = sum_j gradW_ij, Q = sum_j gradW_ij . gradW_ij over a particle with a
 * full rest-lattice neighbourhood and beta = 2 (m dt / rho0)^2. */
double orc_pci_delta(const orc_cfg *c) {
  double s = c->spacing, r = c->support;
  double m = c->mass > 0.0 ? c->mass : c->rho0 / orc_lattice_sum(c);
  double dt = base_dt(c);
  int K = (int)ceil(r / s) + 1;
  double S[3] = {0.0, 0.0, 0.0}, Q = 0.0;
  for (int k = -K; k <= K; ++k)
    for (int j = -K; j <= K; ++j)
      for (int i = -K; i <= K; ++i) {
        if (i == 0 && j == 0 && k == 0) continue;
        double xij[3] = {-i * s, -j * s, -k * s};   /* particle at the origin, j at +(i,j,k)s */
        double d = sqrt(xij[0] * xij[0] + xij[1] * xij[1] + xij[2] * xij[2]);
        if (d >= r) continue;
        double g[3];
        grad_w(c, xij, d, g);
        S[0] += g[0]; S[1] += g[1]; S[2] += g[2];
        Q += g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
      }
  double beta = 2.0 * (m * dt / c->rho0) * (m * dt / c->rho0);
  return -1.0 / (beta * (-(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]) - Q));
}

static void coords_of_key(const orc_info *I, uint32_t k, int32_t b[3]) {
  b[0] = (int32_t)(k % (uint32_t)I->nc[0]);
  uint32_t t = k / (uint32_t)I->nc[0];
  b[1] = (int32_t)(t % (uint32_t)I->nc[1]);
  b[2] = (int32_t)(t / (uint32_t)I->nc[1]);
}
static int in_grid(const orc_info *I, const int32_t q[3]) {
  return q[0] >= 0 && q[1] >= 0 && q[2] >= 0 && q[0] < I->nc[0] && q[1] < I->nc[1] &&
         q[2] < I->nc[2];
}

/* Section 5, "Extra Correction Iterations": regions 1 and 2 grow by a few
 * block layers before a major step, so fast particles stay in them. */
static void dilate_info(const orc_info *I, const uint8_t *in, uint8_t *out, int level,
                        int layers) {
  for (int32_t z = 0; z < I->nc[2]; ++z)
    for (int32_t y = 0; y < I->nc[1]; ++y)
      for (int32_t x = 0; x < I->nc[0]; ++x) {
        int32_t b[3] = {x, y, z};
        uint32_t k = key_of(I, b);
        uint8_t l = in[k];
        if (l != ORC_EMPTY_BLOCK && l > level) {
          int hit = 0;
          for (int dz = -layers; dz <= layers && !hit; ++dz)
            for (int dy = -layers; dy <= layers && !hit; ++dy)
              for (int dx = -layers; dx <= layers && !hit; ++dx) {
                int32_t q[3] = {x + dx, y + dy, z + dz};
                if (in_grid(I, q) && in[key_of(I, q)] == level) hit = 1;
              }
          if (hit) l = (uint8_t)level;
        }
        out[k] = l;
      }
}
void orc_pci_dilate(const orc_cfg *c, const uint8_t *in, uint8_t *out, int level, int layers) {
  orc_info I;
  orc_derive(c, &I);
  dilate_info(&I, in, out, level, layers);
}

/* Figure "regions": observed blocks border a region with a smaller step. */
static void observed_info(const orc_info *I, const uint8_t *lvl, uint8_t *ob) {
  for (int64_t k = 0; k < I->nblocks; ++k) {
    ob[k] = 0;
    if (lvl[k] == ORC_EMPTY_BLOCK) continue;
    int32_t b[3];
    coords_of_key(I, (uint32_t)k, b);
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          int32_t q[3] = {b[0] + dx, b[1] + dy, b[2] + dz};
          if (in_grid(I, q) && lvl[key_of(I, q)] < lvl[k]) ob[k] = 1;
        }
  }
}
void orc_pci_observed(const orc_cfg *c, const uint8_t *lvl, uint8_t *ob) {
  orc_info I;
  orc_derive(c, &I);
  observed_info(&I, lvl, ob);
}

/* a13: Eq. 2 and Eq. 3 per block (Eq. 1 omitted, alpha = 1 via the
 * configuration), dilation of regions 1 then 2, R_min, observed blocks. */
void orc_pci_regions(const orc_cfg *c, int32_t n, const uint32_t *key, const float *vel,
                     const float *acc, uint8_t *raw, uint8_t *lvl, uint8_t *ob) {
  orc_info I;
  orc_derive(c, &I);
  uint8_t *t1 = (uint8_t *)malloc((size_t)I.nblocks), *t2 = (uint8_t *)malloc((size_t)I.nblocks);
  orc_block_levels(c, n, key, vel, acc, raw);
  dilate_info(&I, raw, t1, 0, c->expand_layers);
  dilate_info(&I, t1, t2, 1, c->expand_layers);
  orc_rmin(c, t2, lvl);
  observed_info(&I, lvl, ob);
  free(t1); free(t2);
}

/* a14: neighbours of sorted particle i within the list radius, found in the
 * blocks up to `rings` layers around its block of the stored grid. */
static int32_t pci_list_one(const orc_info *I, int32_t i, const float *pos,
                            const uint32_t *cell_start, const uint32_t *key, const float *wpos,
                            const uint32_t *wcell_start, int32_t rings, int32_t cap,
                            uint32_t *out) {
  int32_t b[3], cnt = 0;
  coords_of_key(I, key[i], b);
  const float *pi = pos + 3 * (int64_t)i;
  for (int pass = 0; pass < 2; ++pass) {
    const uint32_t *st = pass == 0 ? cell_start : wcell_start;
    const float *P = pass == 0 ? pos : wpos;
    if (!st) continue;
    for (int dz = -rings; dz <= rings; ++dz)
      for (int dy = -rings; dy <= rings; ++dy)
        for (int dx = -rings; dx <= rings; ++dx) {
          int32_t q[3] = {b[0] + dx, b[1] + dy, b[2] + dz};
          if (!in_grid(I, q)) continue;
          uint32_t k = key_of(I, q);
          for (uint32_t j = st[k]; j < st[k + 1]; ++j) {
            if (pass == 0 && (int32_t)j == i) continue;
            if (!near_f(pi, P + 3 * (int64_t)j, I->r2l)) continue;
            if (cnt >= cap) return -1;
            out[cnt++] = pass == 0 ? j : (ORC_WALL_BIT | j);
          }
        }
  }
  return cnt;
}

int orc_pci_lists(const orc_cfg *c, int32_t n, const float *pos, const uint32_t *cell_start,
                  const uint32_t *key, int32_t nw, const float *wpos,
                  const uint32_t *wcell_start, const uint8_t *want, const uint8_t *rings,
                  int32_t cap, uint32_t *nbr, int32_t *nnb) {
  orc_info I;
  if (orc_derive(c, &I)) return ORC_E_INVALID;
  int status = ORC_OK;
#pragma omp parallel for schedule(dynamic, 64)
  for (int32_t i = 0; i < n; ++i) {
    if (want && !want[i]) continue;
    int32_t k = pci_list_one(&I, i, pos, cell_start, key, wpos, nw > 0 ? wcell_start : NULL,
                             rings ? rings[i] : 1, cap, nbr + (int64_t)i * cap);
    if (k < 0) {
#pragma omp atomic write
      status = ORC_E_CAPACITY;
      k = 0;
    }
    nnb[i] = k;
  }
  return status;
}

static const double *pci_other(const double *x, const double *wx, uint32_t j) {
  return (j & ORC_WALL_BIT) ? wx + 3 * (int64_t)(j & ~ORC_WALL_BIT) : x + 3 * (int64_t)j;
}

void orc_pci_density(const orc_cfg *c, int32_t n, const double *xs, const double *wx,
                     const uint32_t *nbr, const int32_t *nnb, const uint8_t *which,
                     double *rho) {
  int32_t cap = c->nbr_cap;
  double m = c->mass > 0.0 ? c->mass : c->rho0 / orc_lattice_sum(c);
#pragma omp parallel for schedule(dynamic, 64)
  for (int32_t i = 0; i < n; ++i) {
    if (which && !which[i]) continue;
    const double *xi = xs + 3 * (int64_t)i;
    double sum = orc_kernel_W(c, 0.0);
    const uint32_t *L = nbr + (int64_t)i * cap;
    for (int32_t k = 0; k < nnb[i]; ++k) {
      const double *xj = pci_other(xs, wx, L[k]);
      double d0 = xi[0] - xj[0], d1 = xi[1] - xj[1], d2 = xi[2] - xj[2];
      sum += orc_kernel_W(c, sqrt(d0 * d0 + d1 * d1 + d2 * d2));
    }
    rho[i] = m * sum;
  }
}

void orc_pci_pressure_force(const orc_cfg *c, int32_t n, const double *xs, const double *wx,
                            const double *p, const double *rho, const uint32_t *nbr,
                            const int32_t *nnb, const uint8_t *which, double *fp) {
  orc_pci_pressure_force_terms(c, n, xs, wx, p, rho, nbr, nnb, which, fp, NULL);
}

void orc_pci_pressure_force_terms(const orc_cfg *c, int32_t n, const double *xs,
                                  const double *wx, const double *p, const double *rho,
                                  const uint32_t *nbr, const int32_t *nnb, const uint8_t *which,
                                  double *fp, double *tsum) {
  int32_t cap = c->nbr_cap;
  double m = c->mass > 0.0 ? c->mass : c->rho0 / orc_lattice_sum(c);
#pragma omp parallel for schedule(dynamic, 64)
  for (int32_t i = 0; i < n; ++i) {
    if (which && !which[i]) continue;
    const double *xi = xs + 3 * (int64_t)i;
    double pi = p[i] / (rho[i] * rho[i]);
    double a[3] = {0.0, 0.0, 0.0}, ts = 0.0;
    const uint32_t *L = nbr + (int64_t)i * cap;
    for (int32_t k = 0; k < nnb[i]; ++k) {
      uint32_t j = L[k];
      const double *xj = pci_other(xs, wx, j);
      double xij[3] = {xi[0] - xj[0], xi[1] - xj[1], xi[2] - xj[2]};
      double d = sqrt(xij[0] * xij[0] + xij[1] * xij[1] + xij[2] * xij[2]);
      if (!(d > 0.0) || d >= c->support) continue;
      double pj = (j & ORC_WALL_BIT) ? pi : p[j] / (rho[j] * rho[j]);
      double g[3];
      grad_w(c, xij, d, g);
      for (int e = 0; e < 3; ++e) a[e] -= m * (pi + pj) * g[e];
      ts += fabs(m * (pi + pj)) * sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    }
    for (int e = 0; e < 3; ++e) fp[3 * (int64_t)i + e] = a[e];
    if (tsum) tsum[i] = ts;
  }
}

void orc_pci_nonpressure(const orc_cfg *c, int32_t n, const double *x, const double *v,
                         const double *wx, const uint32_t *nbr, const int32_t *nnb,
                         const uint8_t *which, double *fvg) {
  int32_t cap = c->nbr_cap;
  double m = c->mass > 0.0 ? c->mass : c->rho0 / orc_lattice_sum(c);
  double nu = c->visc_alpha * c->h * c->c0 / c->rho0;
  double eps_h2 = c->visc_eps * c->h * c->h;
#pragma omp parallel for schedule(dynamic, 64)
  for (int32_t i = 0; i < n; ++i) {
    if (which && !which[i]) continue;
    const double *xi = x + 3 * (int64_t)i, *vi = v + 3 * (int64_t)i;
    double a[3] = {c->g[0], c->g[1], c->g[2]};
    const uint32_t *L = nbr + (int64_t)i * cap;
    for (int32_t k = 0; k < nnb[i]; ++k) {
      uint32_t j = L[k];
      const double *xj = pci_other(x, wx, j);
      double vj[3] = {0.0, 0.0, 0.0};          /* walls are at rest */
      if (!(j & ORC_WALL_BIT))
        for (int e = 0; e < 3; ++e) vj[e] = v[3 * (int64_t)j + e];
      double xij[3] = {xi[0] - xj[0], xi[1] - xj[1], xi[2] - xj[2]};
      double d = sqrt(xij[0] * xij[0] + xij[1] * xij[1] + xij[2] * xij[2]);
      if (!(d > 0.0) || d >= c->support) continue;
      double vx = (vi[0] - vj[0]) * xij[0] + (vi[1] - vj[1]) * xij[1] + (vi[2] - vj[2]) * xij[2];
      if (vx >= 0.0) continue;                  /* only approaching pairs are damped */
      double pi_ij = -nu * vx / (d * d + eps_h2);
      double g[3];
      grad_w(c, xij, d, g);
      for (int e = 0; e < 3; ++e) a[e] -= m * pi_ij * g[e];
    }
    for (int e = 0; e < 3; ++e) fvg[3 * (int64_t)i + e] = a[e];
  }
}

/* Figure "iterations" (its image is not in the text we work from): a
 * schedule that meets every stated constraint.  Row 1 holds all regions in
 * every column; the first column's row 2 holds all regions again; region 1
 * gets three rows per minor step, region 2 three rows per two minor steps,
 * regions 3 and 4 fewer per major step (12, 6, 5, 5). */
uint32_t orc_pci_turn(int32_t col, int32_t row) {
  static const uint32_t table[3][4] = {
      {0xF, 0xF, 0xF, 0xF},   /* row 1: R1 R2 R3 R4 */
      {0xF, 0x1, 0x3, 0x1},   /* row 2 */
      {0x1, 0x1, 0x1, 0x1},   /* row 3: R1 */
  };
  if (row < 1 || row > 3 || col < 0 || col > 3) return 0u;
  return table[row - 1][col];
}

int32_t orc_pci_region_validity(int32_t region, int32_t major_len) {
  /* Section 5, neighbourhood updates: R1 every minor step, R2 every second,
   * R3 and R4 at the next major step. */
  return region <= 2 ? region : major_len;
}
#define region_validity orc_pci_region_validity

/* Algorithm 3, the loop's control (C5-C6), taken apart from the physics so
 * that each branch can be driven on its own. */
void orc_pci_ctl_init(const orc_cfg *c, orc_pci_ctl *k) {
  memset(k, 0, sizeof(*k));
  k->iter = 1;
  k->row = 1;
  k->min_iter = c->it_min;
  k->global = 1;
}

int orc_pci_ctl_more(const orc_cfg *c, const orc_pci_ctl *k, double errmax) {
  return (k->iter <= k->min_iter || errmax >= c->eta) && k->iter <= c->it_max;
}

uint32_t orc_pci_ctl_turn(const orc_pci_ctl *k, int32_t col, int32_t standard) {
  if (standard) return 0xFu;
  return k->global ? orc_pci_turn(col, k->row) : 0u;
}

int orc_pci_ctl_after(const orc_cfg *c, orc_pci_ctl *k, int32_t standard, double errmax,
                      double avg) {
  if (k->global) ++k->global_iters;
  ++k->iter;
  ++k->row;
  /* extra iterations start once the three scheduled rows are done */
  if (!(errmax >= c->eta && k->iter > 3)) return ORC_CTL_KEEP;
  ++k->min_iter;
  if (standard) return ORC_CTL_KEEP;
  if (avg >= c->eta_T) {                   /* global error: restart the schedule */
    int act = ORC_CTL_KEEP;
    if (!k->global) {                      /* abandon the local phase */
      act = ORC_CTL_RESTORE;
      ++k->reverts;
      k->local_off = 1;
    }
    k->global = 1;
    k->row = 1;
    ++k->resets;
    return act;
  }
  if (k->local_off) {                      /* the step's one local phase has */
    k->row = 1;                            /* failed: global restarts from here */
    ++k->resets;
    return ORC_CTL_KEEP;
  }
  if (k->global) {                         /* local corrections on S_e */
    k->global = 0;
    k->local_iters = 0;
    return ORC_CTL_BACKUP;
  }
  if (++k->local_iters >= c->local_fail) { /* local phase failed */
    k->global = 1;
    k->local_off = 1;
    k->row = 1;
    ++k->reverts;
    return ORC_CTL_RESTORE;
  }
  return ORC_CTL_KEEP;
}

static void permute_d(double *a, const uint32_t *perm, int32_t n, int w, double *tmp) {
  for (int32_t i = 0; i < n; ++i)
    for (int e = 0; e < w; ++e) tmp[(int64_t)w * i + e] = a[(int64_t)w * perm[i] + e];
  memcpy(a, tmp, sizeof(double) * (size_t)w * (size_t)n);
}
static void permute_u32(uint32_t *a, const uint32_t *perm, int32_t n, uint32_t *tmp) {
  for (int32_t i = 0; i < n; ++i) tmp[i] = a[perm[i]];
  memcpy(a, tmp, sizeof(uint32_t) * (size_t)n);
}

static int pci_standard(const orc_cfg *c) { return c->mode != ORC_MODE_RTS; }

/* Algorithm 2, major-step set-up: grid at block edge e, regions, flags. */
static int pci_major_begin(const orc_cfg *c, const orc_info *I, orc_pci_state *s) {
  int32_t n = s->n;
  size_t nn = (size_t)(n > 0 ? n : 1);
  float *pf = (float *)malloc(sizeof(float) * 3 * nn);
  for (int64_t k = 0; k < 3 * (int64_t)n; ++k) pf[k] = (float)s->x[k];
  uint32_t *key = (uint32_t *)calloc(nn, sizeof(uint32_t));
  uint32_t *perm = (uint32_t *)calloc(nn, sizeof(uint32_t));
  for (int32_t i = 0; i < n; ++i) {
    int32_t b[3];
    block_coords(I, pf + 3 * (int64_t)i, b);
    key[i] = key_of(I, b);
  }
  if (orc_sort(I->nblocks, n, key, perm, s->cell_start)) {
    free(pf); free(key); free(perm);
    return ORC_E_INVALID;
  }
  double *td = (double *)malloc(sizeof(double) * 3 * nn);
  uint32_t *tw = (uint32_t *)malloc(sizeof(uint32_t) * nn);
  permute_d(s->x, perm, n, 3, td);
  permute_d(s->v, perm, n, 3, td);
  permute_d(s->fvg, perm, n, 3, td);
  permute_d(s->fp, perm, n, 3, td);
  permute_d(s->p, perm, n, 1, td);
  permute_d(s->rho, perm, n, 1, td);
  permute_d(s->err, perm, n, 1, td);
  permute_u32(s->id, perm, n, tw);
  for (int32_t i = 0; i < n; ++i) s->key[i] = key[perm[i]];
  /* block maxima of the predicted velocity and the total acceleration of
   * the last minor step, then the regions */
  float *vf = (float *)malloc(sizeof(float) * 3 * nn), *af = (float *)malloc(sizeof(float) * 3 * nn);
  for (int64_t k = 0; k < 3 * (int64_t)n; ++k) {
    vf[k] = (float)s->v[k];
    af[k] = (float)(s->fvg[k] + s->fp[k]);
  }
  uint8_t *raw = (uint8_t *)malloc((size_t)I->nblocks);
  orc_pci_regions(c, n, s->key, vf, af, raw, s->blk_level, s->blk_ob);
  int32_t len = pci_standard(c) ? 1 : s->major_len;
  for (int32_t i = 0; i < n; ++i) {
    s->region[i] = (int32_t)s->blk_level[s->key[i]] + 1;
    s->validity[i] = region_validity(s->region[i], len);
    s->compute[i] = 1;
  }
  free(raw); free(vf); free(af);
  free(pf); free(key); free(perm); free(td); free(tw);
  return ORC_OK;
}

int orc_pci_major_begin(const orc_cfg *c, orc_pci_state *s) {
  orc_info I;
  if (orc_derive(c, &I)) return ORC_E_INVALID;
  return pci_major_begin(c, &I, s);
}

/* blocks holding a particle of S_e, with their 26 neighbours */
static void mark_near_se(const orc_info *I, const orc_pci_state *s, uint8_t *near) {
  memset(near, 0, (size_t)I->nblocks);
  for (int32_t i = 0; i < s->n; ++i) {
    if (!s->in_se[i]) continue;
    int32_t b[3];
    coords_of_key(I, s->key[i], b);
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          int32_t q[3] = {b[0] + dx, b[1] + dy, b[2] + dz};
          if (in_grid(I, q)) near[key_of(I, q)] = 1;
        }
  }
}

/* Adaptive base step (the paper leaves adjusting the PCISPH base step in
 * the manner of global adaptive PCISPH to future work).  Reading taken here:
 * the correction effort of the major step just ended steers the step (an
 * overrun of global_limit or of shrink_iters shrinks it, minor steps that all
 * converged within grow_iters iterations grow it); the Eq. 2-3 limits of the fastest particle
 * cap it, Eq. 3 with beta_2 since beta_1 = infinity bounds nothing. */
static double pci_dt_lo(const orc_cfg *c) { return c->dt_min > 0.0 ? c->dt_min : 0.25 * c->dt_base; }

double orc_pci_next_dt(const orc_cfg *c, double dt, int32_t peak_iters, int32_t excess,
                       float v2max, float a2max) {
  const int32_t grow_at = c->grow_iters > 0 ? c->grow_iters : c->it_min;
  const int32_t shrink_at = c->shrink_iters > 0 ? c->shrink_iters : c->it_min;
  const double lo = pci_dt_lo(c);
  const double hi = c->dt_max > 0.0 ? c->dt_max : 4.0 * c->dt_base;
  double next = dt;
  if (excess || peak_iters > shrink_at)
    next = dt * c->shrink;
  else if (peak_iters <= grow_at)
    next = dt * c->grow;
  if (next > hi) next = hi;
  const double r = r_crit(c);
  if (v2max > 0.0f) {
    const double b = c->alpha_rts * c->beta2 * r / sqrt((double)v2max);    /* Eq. 3, beta_2 */
    if (next > b) next = b;
  }
  if (a2max > 0.0f) {
    const double b = c->lambda_f * sqrt(r / sqrt((double)a2max));          /* Eq. 2 */
    if (next > b) next = b;
  }
  if (next < lo) next = lo;
  return next;
}

/* Section 5, extra iterations: a minor step with more than global_limit
 * global iterations ends its major step early and shortens the following
 * major steps to two minor steps, until short_majors major steps in a row
 * pass without such a minor step. */
int orc_pci_major_length(const orc_cfg *c, orc_pci_state *s, int32_t global_iters,
                         int32_t standard) {
  s->minor_in_major += 1;
  s->last_early_end = 0;
  if (!standard && global_iters > c->global_limit) {
    s->major_excess = 1;
    if (s->minor_in_major < s->major_len) s->last_early_end = 1;
  }
  if (s->minor_in_major < s->major_len && !s->last_early_end) return 0;
  s->minor_in_major = 0;
  if (!standard) {
    if (s->major_excess) {
      s->major_len = 2 < c->n_minor ? 2 : c->n_minor;
      s->clean_majors = 0;
    } else if (s->major_len < c->n_minor && ++s->clean_majors >= c->short_majors) {
      s->major_len = c->n_minor;
      s->clean_majors = 0;
    }
  }
  return 1;
}

/* Section 5, neighbourhood updates: a particle that now needs a smaller
 * step marks its block and the neighbouring blocks to take it. */
int orc_pci_smaller_steps(const orc_cfg *c, int32_t n, const uint32_t *key, const float *vel,
                          const float *acc, int32_t major_len, int32_t *region,
                          int32_t *validity, uint8_t *compute, uint8_t *blk_level,
                          uint8_t *blk_ob) {
  orc_info I;
  if (orc_derive(c, &I)) return 0;
  uint8_t *nl = (uint8_t *)malloc((size_t)I.nblocks);
  memcpy(nl, blk_level, (size_t)I.nblocks);
  int changed = 0;
  for (int32_t i = 0; i < n; ++i) {
    const float v2 = norm2f(vel + 3 * (int64_t)i), a2 = norm2f(acc + 3 * (int64_t)i);
    /* the largest level (region - 1) whose Eq. 2-3 bounds the particle meets */
    int l = 0;
    while (l + 1 <= I.lmax && v2 <= I.TV[l + 1] && a2 <= I.TA[l + 1]) ++l;
    if (l >= region[i] - 1) continue;
    int32_t b[3];
    coords_of_key(&I, key[i], b);
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          int32_t q[3] = {b[0] + dx, b[1] + dy, b[2] + dz};
          if (!in_grid(&I, q)) continue;
          uint32_t kq = key_of(&I, q);
          if (nl[kq] != ORC_EMPTY_BLOCK && nl[kq] > l) { nl[kq] = (uint8_t)l; changed = 1; }
        }
  }
  if (changed) {
    for (int32_t i = 0; i < n; ++i) {
      int32_t r = (int32_t)nl[key[i]] + 1;
      if (r < region[i]) {
        region[i] = r;
        compute[i] = 1;
        validity[i] = region_validity(r, major_len);
      }
    }
    memcpy(blk_level, nl, (size_t)I.nblocks);
    observed_info(&I, blk_level, blk_ob);
  }
  free(nl);
  return changed;
}

int orc_pci_step(const orc_cfg *c_in, orc_pci_state *s) {
  /* this major step's base step: the adapted one once there is one */
  orc_cfg cfg_now = *c_in;
  if (s->dt_cur > 0.0) cfg_now.dt_base = s->dt_cur;
  const orc_cfg *c = &cfg_now;
  orc_info I;
  if (orc_derive(c, &I)) return ORC_E_INVALID;
  int32_t n = s->n;
  size_t nn = (size_t)(n > 0 ? n : 1);
  const int standard = pci_standard(c);
  if (s->major_len <= 0) s->major_len = c->n_minor;
  if (standard) s->major_len = 1;
  const int adapt = !standard && c_in->adapt_dt && s->snap && s->snap_id;
  if (s->minor_in_major == 0) {
    if (adapt) {                   /* the state the major step starts from */
      memcpy(s->snap, s->x, sizeof(double) * 3 * nn);
      memcpy(s->snap + 3 * nn, s->v, sizeof(double) * 3 * nn);
      memcpy(s->snap + 6 * nn, s->fvg, sizeof(double) * 3 * nn);
      memcpy(s->snap + 9 * nn, s->fp, sizeof(double) * 3 * nn);
      memcpy(s->snap + 12 * nn, s->p, sizeof(double) * nn);
      memcpy(s->snap + 13 * nn, s->rho, sizeof(double) * nn);
      memcpy(s->snap + 14 * nn, s->err, sizeof(double) * nn);
      memcpy(s->snap_id, s->id, sizeof(uint32_t) * nn);
      s->snap_t = s->t;
      s->snap_steps = s->minor_steps;
      s->snap_major_len = s->major_len;
      s->snap_clean = s->clean_majors;
    }
    int st = pci_major_begin(c, &I, s);
    if (st) return st;
    s->major_excess = 0;
    s->peak_iters = 0;
  }
  const int32_t col = s->minor_in_major;
  const double dt = I.dt_base, rho0 = c->rho0, eta = c->eta;
  const int32_t cap = c->nbr_cap;

  /* S1: lists of particles whose validity ran out (Section 5,
   * neighbourhood updates), two block layers for region 1 */
  float *pf = (float *)malloc(sizeof(float) * 3 * nn);
  float *wf = (float *)malloc(sizeof(float) * 3 * (size_t)(s->nw > 0 ? s->nw : 1));
  for (int64_t k = 0; k < 3 * (int64_t)n; ++k) pf[k] = (float)s->x[k];
  for (int64_t k = 0; k < 3 * (int64_t)s->nw; ++k) wf[k] = (float)s->wx[k];
  uint8_t *rings = (uint8_t *)malloc(nn);
  int32_t lists = 0;
  const int32_t two = c->two_ring_levels > 0 ? c->two_ring_levels : 1;
  for (int32_t i = 0; i < n; ++i) {
    rings[i] = (uint8_t)((!standard && s->region[i] <= two) ? 2 : 1);
    lists += s->compute[i] ? 1 : 0;
  }
  int st = orc_pci_lists(c, n, pf, s->cell_start, s->key, s->nw, wf, s->wcell_start, s->compute,
                         rings, cap, s->nbr, s->nnb);
  free(pf); free(wf); free(rings);
  if (st) return st;

  /* S2: non-pressure forces of the same particles; S3: p = 0, F^p = 0 */
  orc_pci_nonpressure(c, n, s->x, s->v, s->wx, s->nbr, s->nnb, s->compute, s->fvg);
  for (int32_t i = 0; i < n; ++i) {
    s->p[i] = 0.0;
    s->fp[3 * (int64_t)i] = s->fp[3 * (int64_t)i + 1] = s->fp[3 * (int64_t)i + 2] = 0.0;
    s->in_se[i] = 0;
  }

  /* S4: Algorithm 3 */
  double *xs = (double *)malloc(sizeof(double) * 3 * nn);
  double *p_backup = (double *)calloc(nn, sizeof(double));
  uint8_t *dens = (uint8_t *)malloc(nn), *forc = (uint8_t *)malloc(nn);
  uint8_t *near = (uint8_t *)malloc((size_t)I.nblocks);
  memset(near, 0, (size_t)I.nblocks);
  orc_pci_ctl k;
  orc_pci_ctl_init(c, &k);
  int64_t ev_d = 0, ev_f = 0;
  double errmax = INFINITY, avg = 0.0;
  s->trace_len = 0;
  while (orc_pci_ctl_more(c, &k, errmax)) {
    /* C1: predicted velocity and position of every particle */
    for (int32_t i = 0; i < n; ++i)
      for (int e = 0; e < 3; ++e) {
        int64_t q = 3 * (int64_t)i + e;
        double vs = s->v[q] + dt * (s->fvg[q] + s->fp[q]);
        xs[q] = s->x[q] + dt * vs;
      }
    /* the particles that have the turn */
    const uint32_t turn = orc_pci_ctl_turn(&k, col, standard);
    const int32_t it_row = k.row, it_global = k.global, it_no = k.iter;
    int32_t nd = 0, nf = 0;
    for (int32_t i = 0; i < n; ++i) {
      int t = (turn >> (s->region[i] - 1)) & 1u;
      int ob = s->blk_ob[s->key[i]] || near[s->key[i]];
      dens[i] = (uint8_t)(t || s->in_se[i] || ob);
    }
    /* C2: predicted density, its error, pressure update */
    orc_pci_density(c, n, xs, s->wx, s->nbr, s->nnb, dens, s->rho);
    for (int32_t i = 0; i < n; ++i) {
      if (!dens[i]) continue;
      ++nd;
      s->err[i] = (s->rho[i] - rho0) / rho0;
      double pn = s->p[i] + I.delta * (s->rho[i] - rho0);
      s->p[i] = pn > 0.0 ? pn : 0.0;
    }
    /* C3: S_e gains the particles still over half the allowed error; the
     * blocks around them join the observed set */
    for (int32_t i = 0; i < n; ++i)
      if (dens[i] && s->err[i] > 0.5 * eta) s->in_se[i] = 1;
    mark_near_se(&I, s, near);
    /* C4: pressure acceleration of the particles with the turn and of the
     * updated S_e */
    for (int32_t i = 0; i < n; ++i)
      forc[i] = (uint8_t)(((turn >> (s->region[i] - 1)) & 1u) || s->in_se[i]);
    orc_pci_pressure_force(c, n, xs, s->wx, s->p, s->rho, s->nbr, s->nnb, forc, s->fp);
    for (int32_t i = 0; i < n; ++i) nf += forc[i];
    ev_d += nd;
    ev_f += nf;
    /* C5: errors over the fluid (particles not evaluated keep their last) */
    errmax = 0.0;
    double sum = 0.0;
    for (int32_t i = 0; i < n; ++i) {
      double e = s->err[i] > 0.0 ? s->err[i] : 0.0;
      if (e > errmax) errmax = e;
      sum += e;
    }
    avg = n > 0 ? sum / n : 0.0;
    /* C6: extra iterations after the three scheduled ones */
    const int act = orc_pci_ctl_after(c, &k, standard, errmax, avg);
    if (act == ORC_CTL_BACKUP) memcpy(p_backup, s->p, sizeof(double) * nn);
    if (act == ORC_CTL_RESTORE) memcpy(s->p, p_backup, sizeof(double) * nn);
    if (s->trace && s->trace_len < s->trace_cap) {
      orc_pci_iter_rec *r = &s->trace[s->trace_len];
      int32_t nse = 0;
      for (int32_t i = 0; i < n; ++i) nse += s->in_se[i];
      r->iter = it_no;
      r->row = it_row;
      r->global = it_global;
      r->turn = turn;
      r->action = act;
      r->n_density = nd;
      r->n_force = nf;
      r->n_se = nse;
      r->errmax = errmax;
      r->avg = avg;
      if (s->trace_p)
        memcpy(s->trace_p + (int64_t)s->trace_len * n, s->p, sizeof(double) * (size_t)n);
      if (s->trace_e)
        for (int32_t i = 0; i < n; ++i)
          s->trace_e[(int64_t)s->trace_len * n + i] = dens[i] ? s->err[i] : NAN;
      s->trace_len += 1;
    }
  }
  const int32_t iter = k.iter, global_iters = k.global_iters;
  const int32_t resets = k.resets, reverts = k.reverts;
  free(xs); free(p_backup); free(dens); free(forc); free(near);

  /* S5: new velocity and position (symplectic Euler) */
  for (int64_t k = 0; k < 3 * (int64_t)n; ++k) {
    s->v[k] += dt * (s->fvg[k] + s->fp[k]);
    s->x[k] += dt * s->v[k];
  }
  /* S6: validity */
  for (int32_t i = 0; i < n; ++i) {
    s->validity[i] -= 1;
    if (s->validity[i] <= 0) {
      s->compute[i] = 1;
      s->validity[i] = region_validity(s->region[i], s->major_len);
    } else {
      s->compute[i] = 0;
    }
  }
  /* S7: a particle that now needs a smaller step takes its block and the 26
   * around it to that step */
  if (!standard) {
    float *vf = (float *)malloc(sizeof(float) * 3 * nn), *af = (float *)malloc(sizeof(float) * 3 * nn);
    for (int64_t q = 0; q < 3 * (int64_t)n; ++q) {
      vf[q] = (float)s->v[q];
      af[q] = (float)(s->fvg[q] + s->fp[q]);
    }
    orc_pci_smaller_steps(c, n, s->key, vf, af, s->major_len, s->region, s->validity, s->compute,
                          s->blk_level, s->blk_ob);
    free(vf);
    free(af);
  }

  /* statistics and the major-step length (Section 5, extra iterations) */
  s->last_iters = iter - 1;
  s->last_global_iters = global_iters;
  s->last_resets = resets;
  s->last_reverts = reverts;
  s->last_lists = lists;
  s->evals_density = ev_d;
  s->evals_force = ev_f;
  s->last_errmax = errmax;
  s->last_avg = avg;
  for (int r = 0; r < 4; ++r) s->hist[r] = 0;
  for (int32_t i = 0; i < n; ++i) s->hist[s->region[i] - 1]++;
  if (iter - 1 > s->peak_iters) s->peak_iters = iter - 1;
  s->last_dt = dt;
  s->t += dt;
  s->minor_steps += 1;
  const int ends = orc_pci_major_length(c, s, global_iters, standard);
  if (ends) {
    if (adapt) {
      /* the next major step's base step, from this one's effort and the
       * fastest particle after it */
      float v2m = 0.0f, a2m = 0.0f;
      for (int32_t i = 0; i < n; ++i) {
        float vf[3], af[3];
        for (int e = 0; e < 3; ++e) {
          vf[e] = (float)s->v[3 * (int64_t)i + e];
          af[e] = (float)(s->fvg[3 * (int64_t)i + e] + s->fp[3 * (int64_t)i + e]);
        }
        const float v2 = norm2f(vf), a2 = norm2f(af);
        if (v2 > v2m) v2m = v2;
        if (a2 > a2m) a2m = a2;
      }
      s->last_v2max = v2m;
      s->last_a2max = a2m;
      s->dt_cur = orc_pci_next_dt(c_in, dt, s->peak_iters, s->major_excess, v2m, a2m);
    }
  }
  /* a correction that did not converge: back to the start of the major
   * step, which restarts with half the step */
  s->last_rollback = 0;
  if (adapt && errmax >= eta && dt > pci_dt_lo(c_in)) {
    memcpy(s->x, s->snap, sizeof(double) * 3 * nn);
    memcpy(s->v, s->snap + 3 * nn, sizeof(double) * 3 * nn);
    memcpy(s->fvg, s->snap + 6 * nn, sizeof(double) * 3 * nn);
    memcpy(s->fp, s->snap + 9 * nn, sizeof(double) * 3 * nn);
    memcpy(s->p, s->snap + 12 * nn, sizeof(double) * nn);
    memcpy(s->rho, s->snap + 13 * nn, sizeof(double) * nn);
    memcpy(s->err, s->snap + 14 * nn, sizeof(double) * nn);
    memcpy(s->id, s->snap_id, sizeof(uint32_t) * nn);
    s->t = s->snap_t;
    s->minor_steps = s->snap_steps;
    s->major_len = s->snap_major_len;
    s->clean_majors = s->snap_clean;
    s->minor_in_major = 0;
    const double lo = pci_dt_lo(c_in), half = 0.5 * dt;
    s->dt_cur = half > lo ? half : lo;
    s->rollbacks += 1;
    s->last_rollback = 1;
  }
  for (int64_t k = 0; k < 3 * (int64_t)n; ++k)
    if (!isfinite(s->x[k])) return ORC_E_NUMERICAL;
  return ORC_OK;
}

/* ======================================================================== */
/* Differentiable WCSPH substep and its adjoint (reverse accumulation in     */
/* scatter form: each ordered neighbour pair pushes its partial derivatives  */
/* to both particles).                                                       */
/* ======================================================================== */
static double d2w_shape(double q) { /* d^2 w_shape / dq^2 */
  if (q < 1.0) return -3.0 + 4.5 * q;
  if (q < 2.0) return 1.5 * (2.0 - q);
  return 0.0;
}

typedef struct {
  double *x, *v, *rho, *p;   /* state at the substep's start, and its density and pressure */
  uint32_t *nbr;
  int32_t *nnb;
  int32_t cap;
} diff_frame;

static int diff_lists(const orc_cfg *c, int32_t n, const double *x, int32_t nw, const double *wx,
                      diff_frame *f) {
  ctx_t X;
  if (ctx_open(&X, c, n, x, nw, wx)) return ORC_E_INVALID;
  int st = ctx_lists(&X, NULL);
  f->cap = X.cap;
  memcpy(f->nbr, X.nbr, sizeof(uint32_t) * (size_t)X.cap * (size_t)(n > 0 ? n : 1));
  memcpy(f->nnb, X.nnb, sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  ctx_close(&X);
  return st;
}

/* one forward substep from f->x, f->v (lists, rho, p filled in f) */
static void diff_substep(const orc_cfg *c, const orc_info *I, int32_t n, const double *wx,
                         double B, double alpha, double dt, diff_frame *f, double *x1,
                         double *v1) {
  const double m = I->mass, h = c->h, e = c->visc_eps * h * h, rho0 = c->rho0;
  for (int32_t i = 0; i < n; ++i) {
    const double *xi = f->x + 3 * (int64_t)i;
    double sum = orc_kernel_W(c, 0.0);
    const uint32_t *L = f->nbr + (int64_t)i * f->cap;
    for (int32_t k = 0; k < f->nnb[i]; ++k) {
      const double *xj = pci_other(f->x, wx, L[k]);
      double d0 = xi[0] - xj[0], d1 = xi[1] - xj[1], d2 = xi[2] - xj[2];
      sum += orc_kernel_W(c, sqrt(d0 * d0 + d1 * d1 + d2 * d2));
    }
    f->rho[i] = m * sum;
    f->p[i] = B * (pow(f->rho[i] / rho0, 7.0) - 1.0);
  }
  for (int32_t i = 0; i < n; ++i) {
    const double *xi = f->x + 3 * (int64_t)i, *vi = f->v + 3 * (int64_t)i;
    const double ri = f->rho[i], Pi_ = f->p[i] / (ri * ri);
    double a[3] = {c->g[0], c->g[1], c->g[2]};
    const uint32_t *L = f->nbr + (int64_t)i * f->cap;
    for (int32_t k = 0; k < f->nnb[i]; ++k) {
      const uint32_t j = L[k];
      const int wall = (j & ORC_WALL_BIT) != 0;
      const double *xj = pci_other(f->x, wx, j);
      double vj[3] = {0.0, 0.0, 0.0};
      double coef, nu;
      if (wall) {
        coef = 2.0 * Pi_;
        nu = alpha * h * c->c0 / ri;
      } else {
        for (int d = 0; d < 3; ++d) vj[d] = f->v[3 * (int64_t)j + d];
        const double rj = f->rho[j];
        coef = Pi_ + f->p[j] / (rj * rj);
        nu = 2.0 * alpha * h * c->c0 / (ri + rj);
      }
      double xij[3] = {xi[0] - xj[0], xi[1] - xj[1], xi[2] - xj[2]};
      double r2 = xij[0] * xij[0] + xij[1] * xij[1] + xij[2] * xij[2];
      double r = sqrt(r2);
      if (!(r > 0.0) || r >= c->support) continue;
      double s = (vi[0] - vj[0]) * xij[0] + (vi[1] - vj[1]) * xij[1] + (vi[2] - vj[2]) * xij[2];
      if (s < 0.0) coef += -nu * s / (r2 + e);
      double F = orc_kernel_dWdr(c, r) / r;
      for (int d = 0; d < 3; ++d) a[d] -= m * coef * F * xij[d];
    }
    for (int d = 0; d < 3; ++d) {
      int64_t q = 3 * (int64_t)i + d;
      v1[q] = vi[d] + dt * a[d];
      x1[q] = xi[d] + dt * v1[q];
    }
  }
}

static int diff_forward(const orc_cfg *c, int32_t n, const double *x0, const double *v0,
                        int32_t nw, const double *wx, double B, double alpha, double dt,
                        int32_t n_sub, diff_frame *frames, double *x_out, double *v_out) {
  orc_info I;
  if (orc_derive(c, &I)) return ORC_E_INVALID;
  size_t sz = sizeof(double) * 3 * (size_t)n;
  memcpy(frames[0].x, x0, sz);
  memcpy(frames[0].v, v0, sz);
  for (int32_t k = 0; k < n_sub; ++k) {
    diff_frame *f = &frames[k];
    int st = diff_lists(c, n, f->x, nw, wx, f);
    if (st) return st;
    double *x1 = k + 1 < n_sub ? frames[k + 1].x : x_out;
    double *v1 = k + 1 < n_sub ? frames[k + 1].v : v_out;
    diff_substep(c, &I, n, wx, B, alpha, dt, f, x1, v1);
  }
  return ORC_OK;
}

static diff_frame *frames_new(int32_t n, int32_t n_sub, int32_t cap) {
  diff_frame *fr = (diff_frame *)calloc((size_t)n_sub, sizeof(diff_frame));
  size_t nn = (size_t)(n > 0 ? n : 1);
  for (int32_t k = 0; k < n_sub; ++k) {
    fr[k].x = (double *)malloc(sizeof(double) * 3 * nn);
    fr[k].v = (double *)malloc(sizeof(double) * 3 * nn);
    fr[k].rho = (double *)malloc(sizeof(double) * nn);
    fr[k].p = (double *)malloc(sizeof(double) * nn);
    fr[k].nbr = (uint32_t *)malloc(sizeof(uint32_t) * nn * (size_t)cap);
    fr[k].nnb = (int32_t *)malloc(sizeof(int32_t) * nn);
  }
  return fr;
}
static void frames_free(diff_frame *fr, int32_t n_sub) {
  for (int32_t k = 0; k < n_sub; ++k) {
    free(fr[k].x); free(fr[k].v); free(fr[k].rho); free(fr[k].p); free(fr[k].nbr);
    free(fr[k].nnb);
  }
  free(fr);
}

int orc_diff_run(const orc_cfg *c, int32_t n, const double *x0, const double *v0, int32_t nw,
                 const double *wx, double B, double alpha, double dt, int32_t n_sub,
                 double *x_out, double *v_out) {
  if (n_sub < 1) return ORC_E_INVALID;
  int32_t cap = c->nbr_cap > 0 ? c->nbr_cap : 512;
  diff_frame *fr = frames_new(n, n_sub, cap);
  int st = diff_forward(c, n, x0, v0, nw, wx, B, alpha, dt, n_sub, fr, x_out, v_out);
  frames_free(fr, n_sub);
  return st;
}

int orc_diff_grad(const orc_cfg *c, int32_t n, const double *x0, const double *v0, int32_t nw,
                  const double *wx, double B, double alpha, double dt, int32_t n_sub,
                  const double *xhat, double *loss, double *g_x0, double *g_v0, double *g_B,
                  double *g_alpha) {
  if (n_sub < 1 || n < 1) return ORC_E_INVALID;
  orc_info I;
  if (orc_derive(c, &I)) return ORC_E_INVALID;
  int32_t cap = c->nbr_cap > 0 ? c->nbr_cap : 512;
  diff_frame *fr = frames_new(n, n_sub, cap);
  size_t n3 = 3 * (size_t)n;
  double *xT = (double *)malloc(sizeof(double) * n3), *vT = (double *)malloc(sizeof(double) * n3);
  int st = diff_forward(c, n, x0, v0, nw, wx, B, alpha, dt, n_sub, fr, xT, vT);
  if (st) { frames_free(fr, n_sub); free(xT); free(vT); return st; }
  const double m = I.mass, h = c->h, e = c->visc_eps * h * h, rho0 = c->rho0;
  double L = 0.0;
  double *xb = (double *)calloc(n3, sizeof(double)), *vb = (double *)calloc(n3, sizeof(double));
  for (size_t q = 0; q < n3; ++q) {
    double d = xT[q] - xhat[q];
    L += d * d;
    xb[q] = 2.0 * d / n;
  }
  *loss = L / n;
  double Bb = 0.0, ab_alpha = 0.0;
  double *ab = (double *)malloc(sizeof(double) * n3);
  double *xn = (double *)malloc(sizeof(double) * n3), *vn = (double *)malloc(sizeof(double) * n3);
  double *Pb = (double *)malloc(sizeof(double) * (size_t)n), *rb = (double *)malloc(sizeof(double) * (size_t)n);
  for (int32_t k = n_sub - 1; k >= 0; --k) {
    diff_frame *f = &fr[k];
    /* x' = x + dt v',  v' = v + dt a */
    for (size_t q = 0; q < n3; ++q) {
      double vt = vb[q] + dt * xb[q];
      ab[q] = dt * vt;
      xn[q] = xb[q];
      vn[q] = vt;
    }
    memset(Pb, 0, sizeof(double) * (size_t)n);
    memset(rb, 0, sizeof(double) * (size_t)n);
    /* forces: a_i -= t_ij, t = m c G(x_ij); the upstream gradient of t is -ab_i */
    for (int32_t i = 0; i < n; ++i) {
      const double *xi = f->x + 3 * (int64_t)i, *vi = f->v + 3 * (int64_t)i;
      const double ri = f->rho[i], Pi_ = f->p[i] / (ri * ri);
      const double u[3] = {-ab[3 * (int64_t)i], -ab[3 * (int64_t)i + 1], -ab[3 * (int64_t)i + 2]};
      const uint32_t *Lst = f->nbr + (int64_t)i * f->cap;
      for (int32_t kk = 0; kk < f->nnb[i]; ++kk) {
        const uint32_t j = Lst[kk];
        const int wall = (j & ORC_WALL_BIT) != 0;
        const double *xj = pci_other(f->x, wx, j);
        double vj[3] = {0.0, 0.0, 0.0}, rj = ri, coef, nu;
        if (wall) {
          coef = 2.0 * Pi_;
          nu = alpha * h * c->c0 / ri;
        } else {
          for (int d = 0; d < 3; ++d) vj[d] = f->v[3 * (int64_t)j + d];
          rj = f->rho[j];
          coef = Pi_ + f->p[j] / (rj * rj);
          nu = 2.0 * alpha * h * c->c0 / (ri + rj);
        }
        double x[3] = {xi[0] - xj[0], xi[1] - xj[1], xi[2] - xj[2]};
        double vv[3] = {vi[0] - vj[0], vi[1] - vj[1], vi[2] - vj[2]};
        double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
        double r = sqrt(r2);
        if (!(r > 0.0) || r >= c->support) continue;
        double s = vv[0] * x[0] + vv[1] * x[1] + vv[2] * x[2];
        const int visc = s < 0.0;
        const double den = r2 + e;
        if (visc) coef += -nu * s / den;
        const double q = r / h, sig = 1.0 / (M_PI * h * h * h);
        const double W1 = sig * dw_shape(q) / h, W2 = sig * d2w_shape(q) / (h * h);
        const double F = W1 / r, dF = (W2 * r - W1) / r2;
        const double G[3] = {F * x[0], F * x[1], F * x[2]};
        const double Gu = G[0] * u[0] + G[1] * u[1] + G[2] * u[2];
        const double xu = x[0] * u[0] + x[1] * u[1] + x[2] * u[2];
        double gx[3], gv[3] = {0.0, 0.0, 0.0};
        for (int d = 0; d < 3; ++d) gx[d] = m * coef * (F * u[d] + dF / r * x[d] * xu);
        if (visc) {
          for (int d = 0; d < 3; ++d) {
            const double dcdx = -nu * (vv[d] / den - 2.0 * s * x[d] / (den * den));
            gx[d] += dcdx * m * Gu;
            gv[d] = -nu * x[d] / den * m * Gu;
          }
          const double nub = -s / den * m * Gu;
          ab_alpha += nub * nu / alpha;
          if (wall) {
            rb[i] += nub * (-nu / ri);
          } else {
            rb[i] += nub * (-nu / (ri + rj));
            rb[j] += nub * (-nu / (ri + rj));
          }
        }
        for (int d = 0; d < 3; ++d) {
          xn[3 * (int64_t)i + d] += gx[d];
          vn[3 * (int64_t)i + d] += gv[d];
        }
        if (wall) {
          Pb[i] += 2.0 * m * Gu;
        } else {
          Pb[i] += m * Gu;
          Pb[j] += m * Gu;
          for (int d = 0; d < 3; ++d) {
            xn[3 * (int64_t)j + d] -= gx[d];
            vn[3 * (int64_t)j + d] -= gv[d];
          }
        }
      }
    }
    /* P = p / rho^2, EOS */
    for (int32_t i = 0; i < n; ++i) {
      const double ri = f->rho[i], pi = f->p[i];
      const double pb = Pb[i] / (ri * ri);
      rb[i] += Pb[i] * (-2.0 * pi / (ri * ri * ri));
      rb[i] += pb * 7.0 * B * pow(ri / rho0, 6.0) / rho0;
      Bb += pb * (pow(ri / rho0, 7.0) - 1.0);
    }
    /* density: rho_i = m sum_j W(|x_i - x_j|) */
    for (int32_t i = 0; i < n; ++i) {
      const double *xi = f->x + 3 * (int64_t)i;
      const uint32_t *Lst = f->nbr + (int64_t)i * f->cap;
      for (int32_t kk = 0; kk < f->nnb[i]; ++kk) {
        const uint32_t j = Lst[kk];
        const double *xj = pci_other(f->x, wx, j);
        double x[3] = {xi[0] - xj[0], xi[1] - xj[1], xi[2] - xj[2]};
        double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        if (!(r > 0.0) || r >= c->support) continue;
        const double F = orc_kernel_dWdr(c, r) / r;
        for (int d = 0; d < 3; ++d) {
          const double g = m * F * x[d] * rb[i];
          xn[3 * (int64_t)i + d] += g;
          if (!(j & ORC_WALL_BIT)) xn[3 * (int64_t)j + d] -= g;
        }
      }
    }
    memcpy(xb, xn, sizeof(double) * n3);
    memcpy(vb, vn, sizeof(double) * n3);
  }
  memcpy(g_x0, xb, sizeof(double) * n3);
  memcpy(g_v0, vb, sizeof(double) * n3);
  *g_B = Bb;
  *g_alpha = ab_alpha;
  free(xb); free(vb); free(ab); free(xn); free(vn); free(Pb); free(rb); free(xT); free(vT);
  frames_free(fr, n_sub);
  return ORC_OK;
}
