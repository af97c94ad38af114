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
  /* Level l steps 2^l base steps and is ranked n = l + 1 for beta (Eq. 3):
   *   Eq. 3:  2^l dt |v| / r <= alpha beta_{l+1}  ->  |v|^2 <= TV[l]
   *   Eq. 2:  2^l dt <= lambda_f sqrt(r / |a|)    ->  |a|^2 <= TA[l]   */
  for (int l = 0; l < ORC_MAX_LEVELS; ++l) {
    double dtl = ldexp(o->dt_base, l);
    double b = beta_n(c, l + 1);
    double vl = isinf(b) ? INFINITY : c->alpha_rts * b * r_crit(c) / dtl;
    double al = c->lambda_f * c->lambda_f * r_crit(c) / (dtl * dtl);
    o->TV[l] = (float)(vl * vl);
    o->TA[l] = (float)(al * al);
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
               int32_t *validity, uint8_t *compute) {
  for (int32_t i = 0; i < n; ++i) {
    int32_t bl = blk[key[i]];
    validity[i] -= 1;
    if (validity[i] <= 0 || level[i] != bl) {
      compute[i] = 1;
      level[i] = bl;
      validity[i] = 1 << bl;
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
                              const uint8_t *which, double *acc) {
  double m = X->I.mass, h = c->h;
#pragma omp parallel for schedule(dynamic, 64)
  for (int32_t i = 0; i < X->n; ++i) {
    if (which && !which[i]) continue;
    const double *xi = x + 3 * (int64_t)i, *vi = v + 3 * (int64_t)i;
    double ri = rho[i], pi = p[i];
    double ai[3] = {c->g[0], c->g[1], c->g[2]};
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
    }
    for (int d = 0; d < 3; ++d) acc[3 * (int64_t)i + d] = ai[d];
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
  forces_from_lists(c, &X, x, v, rho, p, wx, which, acc);
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
  orc_flags(n, X.gf.key, lvl, s->level, s->validity, s->compute);

  /* W6-W8 */
  status = ctx_lists(&X, s->compute);
  density_from_lists(c, &X, s->x, s->wx, s->compute, s->rho, s->p);
  double *anew = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
  forces_from_lists(c, &X, s->x, s->v, s->rho, s->p, s->wx, s->compute, anew);

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
  double dt = I->dt_base;
  if (c->mode == ORC_MODE_GLOBAL_ADAPTIVE) {
    double amax2 = 0.0;
    for (int32_t i = 0; i < n; ++i) {
      const double *ai = s->a + 3 * (int64_t)i;
      double a2 = ai[0] * ai[0] + ai[1] * ai[1] + ai[2] * ai[2];
      if (a2 > amax2) amax2 = a2;
    }
    dt = c->lambda_v * r_crit(c) / c->c0;
    if (amax2 > 0.0) {
      double df = c->lambda_f * sqrt(r_crit(c) / sqrt(amax2));
      if (df < dt) dt = df;
    }
  }
  orc_serna_predict(n, s->x, s->v, s->a, dt);
  for (int32_t i = 0; i < n; ++i) s->age[i] += 1;
  s->dt_prev = dt;
  s->t += dt;
  s->step += 1;

  free(vf); free(af); free(lraw); free(lvl); free(anew); free(dtau);
  ctx_close(&X);
  return status;
}
