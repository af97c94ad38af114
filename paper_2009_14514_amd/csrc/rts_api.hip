// C ABI of the RTS library: configuration, workspace carving, state
// transfer, the base-step driver (replayed as HIP graphs) and counters.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>

#include "rts_internal.h"

using namespace rts;

struct rts_ctx {
  rts_config cfg;
  DevParams prm;
  DevPtrs d;
  int cur;
  hipStream_t stream;
  hipStream_t cap_stream;
  hipGraphExec_t gexec[2];
  hipGraph_t graph[2];
  bool graph_ok;
  int64_t ncap, nwcap;
  int grid_wave;     // workgroups of the one-wave-per-block kernels (4 waves each)
  int grid_search;   // workgroups of the search / density kernel
  int grid_force;    // workgroups of the force kernel
  int search_threads;  // threads per search / density workgroup (256, 512)
  int force_lanes;     // force lanes per particle (4, 8)
  bool has_state;
  bool poisoned;
  double mass, B, dt_base;
  // PCISPH schedule state (host side: the correction loop is driven from here)
  int pci_major_len, pci_minor_in_major, pci_clean, pci_excess;
  bool pci_ready;        // the current major step has been set up
  int64_t pci_steps, pci_iters_total;
  double pci_time;
  int32_t pci_last[6];   // iters, global iters, resets, reverts, early end, lists
  double pci_errmax, pci_avg;
  int32_t pci_hist[4];
  // adaptive base step: the last minor step's length, the most iterations
  // of a minor step in this major step, and what a roll-back restores (the
  // particle state itself stays in the sort's source buffers, cur ^ 1,
  // which the minor steps never write)
  double dt_last;
  int pci_peak;
  int32_t pci_rollbacks;
  double snap_time;
  int64_t snap_steps;
  int snap_major_len, snap_clean;
  // fixed base step: the last step's closing kernel has binned the current
  // positions for the next sort (keys, ranks, block counts), so the next
  // step starts with its scan; anything else that sorts, or that replaces
  // the particles, first clears those counts (unbin)
  bool binned;
  int tune_candidates;
  double tune_ms;
  int static_dev;    // device whose static workspace holds this context, or -1
  char *ws;          // workspace base and the bytes the buffer table uses
  size_t ws_used;
  // scenes: a batched context has fixed scene sizes (rts_create_batch);
  // otherwise one scene of whatever rts_set_state gives
  bool batched;
  int32_t n_scenes;
  uint32_t *scene_off;   // n_scenes + 1 caller offsets (host copy)
  int64_t *scene_fill;   // particles written by rts_init_dam_break since the last reset
  bool fresh;            // the state is in caller order: nothing has sorted it yet
  char err[512];
};

// The library's own workspace for callers that cannot allocate device
// memory (rts_create_static): one array per device, held until the process
// ends.  Host code never uses the array's name as an address: each device's
// address comes from hipGetSymbolAddress with that device current.
static __device__ __align__(256) uint8_t scratch[RTS_STATIC_WORKSPACE_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void *g_static_ptr[kMaxDevices];   // device address of `scratch` on each device
bool g_static_busy[kMaxDevices];   // a live context uses that device's array

}  // namespace

namespace {

rts_status fail(rts_ctx *c, rts_status s, const char *fmt, ...) {
  if (c) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(c->err, sizeof(c->err), fmt, ap);
    va_end(ap);
  }
  return s;
}

#define HIP_OK(ctx, expr)                                                                  \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail((ctx), RTS_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

// Cubic spline shape, used on the host for the mass calibration.
double w_shape_d(double q) {
  if (q < 1.0) return 1.0 - 1.5 * q * q + 0.75 * q * q * q;
  if (q < 2.0) {
    double t = 2.0 - q;
    return 0.25 * t * t * t;
  }
  return 0.0;
}

// Sum of W over the cubic lattice around one site, self included: a
// particle in the interior of the rest lattice then has density rho0.
double lattice_w_sum(const rts_config &c) {
  double s = c.spacing, r = c.support;
  double sigma = 1.0 / (M_PI * c.h * c.h * c.h);
  int m = (int)ceil(r / s) + 1;
  double sum = 0.0;
  for (int k = -m; k <= m; ++k)
    for (int j = -m; j <= m; ++j)
      for (int i = -m; i <= m; ++i) {
        double d = s * sqrt((double)(i * i + j * j + k * k));
        if (d < r) sum += sigma * w_shape_d(d / c.h);
      }
  return sum;
}

double r_crit_of(const rts_config &c) { return c.r_crit > 0.0 ? c.r_crit : c.support; }

// Cubic spline shape derivative d w / d q.
double dw_shape_d(double q) {
  if (q < 1.0) return -3.0 * q + 2.25 * q * q;
  if (q < 2.0) {
    double t = 2.0 - q;
    return -0.75 * t * t;
  }
  return 0.0;
}

// The PCISPH pressure coefficient of standard PCISPH (Solenthaler &
// Pajarola), evaluated once over a particle with a full rest-lattice
// neighbourhood: with g_j the kernel gradient towards lattice neighbour j,
// G = sum_j g_j and Q = sum_j |g_j|^2, delta = 1 / (beta (|G|^2 + Q)),
// beta = 2 (m dt / rho0)^2.
double pci_delta(const rts_config &c, double mass, double dt) {
  const double s = c.spacing, r = c.support;
  const int m = (int)ceil(r / s) + 1;
  double G[3] = {0.0, 0.0, 0.0}, Q = 0.0;
  for (int k = -m; k <= m; ++k)
    for (int j = -m; j <= m; ++j)
      for (int i = -m; i <= m; ++i) {
        if (!i && !j && !k) continue;
        const double x[3] = {i * s, j * s, k * s};
        const double d = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        if (d >= r) continue;
        const double f = dw_shape_d(d / c.h) / (M_PI * c.h * c.h * c.h * c.h) / d;
        for (int e = 0; e < 3; ++e) G[e] += f * x[e];
        Q += f * f * d * d;
      }
  const double beta = 2.0 * (mass * dt / c.rho0) * (mass * dt / c.rho0);
  return 1.0 / (beta * (G[0] * G[0] + G[1] * G[1] + G[2] * G[2] + Q));
}

rts_status validate(const rts_config *c, char *msg, size_t cap) {
  if (!c) { snprintf(msg, cap, "config is NULL"); return RTS_E_INVALID; }
  if (c->solver != RTS_WCSPH && c->solver != RTS_PCISPH) {
    snprintf(msg, cap, "unknown solver %d", c->solver);
    return RTS_E_INVALID;
  }
  if (c->mode < 0 || c->mode > 2) { snprintf(msg, cap, "bad mode %d", c->mode); return RTS_E_INVALID; }
  if (c->phase_align != 0 && c->phase_align != 1) {
    snprintf(msg, cap, "phase_align must be 0 or 1");
    return RTS_E_INVALID;
  }
  if (c->nbr_cap < 8 || c->nbr_cap > 4096) {
    snprintf(msg, cap, "nbr_cap must be in [8, 4096]");
    return RTS_E_INVALID;
  }
  if (c->solver == RTS_PCISPH) {
    if (c->mode == RTS_MODE_GLOBAL_ADAPTIVE) {
      snprintf(msg, cap, "PCISPH runs regional (rts) or standard (global_fixed) stepping");
      return RTS_E_UNSUPPORTED;
    }
    if (c->n_levels != 4) { snprintf(msg, cap, "PCISPH has 4 regions"); return RTS_E_INVALID; }
    if (c->n_minor < 1 || c->n_minor > 16 || c->it_min < 1 || c->it_max < c->it_min ||
        c->it_max > 1000 || c->expand_layers < 0 || c->expand_layers > 16 ||
        c->local_fail < 1 || c->global_limit < 1 || c->short_majors < 1) {
      snprintf(msg, cap, "PCISPH schedule parameters out of range");
      return RTS_E_INVALID;
    }
    if (c->two_ring_levels < 0 || c->two_ring_levels > 4) {
      snprintf(msg, cap, "two_ring_levels must be in [0, 4]");
      return RTS_E_INVALID;
    }
    if (!(c->eta > 0 && c->eta_T > 0 && c->dt_base > 0)) {
      snprintf(msg, cap, "PCISPH needs eta, eta_T and dt_base > 0");
      return RTS_E_INVALID;
    }
    if (c->pci_adapt_dt) {
      const double lo = c->pci_dt_min > 0 ? c->pci_dt_min : 0.25 * c->dt_base;
      const double hi = c->pci_dt_max > 0 ? c->pci_dt_max : 4.0 * c->dt_base;
      if (c->pci_adapt_dt != 1 || !(c->pci_grow >= 1.0) || !(c->pci_shrink > 0.0) ||
          !(c->pci_shrink <= 1.0) || !(lo <= c->dt_base && c->dt_base <= hi) ||
          c->delta > 0.0) {
        snprintf(msg, cap, "adaptive base step: need pci_grow >= 1, 0 < pci_shrink <= 1, "
                 "pci_dt_min <= dt_base <= pci_dt_max and delta <= 0");
        return RTS_E_INVALID;
      }
    }
    const double rl = c->r_list > 0 ? c->r_list : c->block_edge;
    if (!(rl >= c->support && rl <= c->block_edge)) {
      snprintf(msg, cap, "r_list must lie in [support, block_edge]");
      return RTS_E_INVALID;
    }
  }
  if (!(c->spacing > 0 && c->h > 0 && c->support > 0 && c->rho0 > 0 && c->c0 > 0)) {
    snprintf(msg, cap, "spacing, h, support, rho0 and c0 must be positive");
    return RTS_E_INVALID;
  }
  if (!(c->support <= 2.0 * c->h * (1.0 + 1e-12))) {
    snprintf(msg, cap, "support %g exceeds the cubic spline's 2h", c->support);
    return RTS_E_INVALID;
  }
  if (!(c->block_edge >= c->support)) {
    snprintf(msg, cap, "block_edge %g must be >= support %g", c->block_edge, c->support);
    return RTS_E_INVALID;
  }
  if (c->gamma != 7.0) { snprintf(msg, cap, "only gamma = 7 is built"); return RTS_E_UNSUPPORTED; }
  if (c->n_levels < 1 || c->n_levels > RTS_MAX_LEVELS) {
    snprintf(msg, cap, "n_levels must be in [1, %d]", RTS_MAX_LEVELS);
    return RTS_E_INVALID;
  }
  // a block's candidates are indexed by 16-bit list entries
  if (c->cand_cap < 32 * kSub || c->cand_cap > 65536 || c->cand_cap % (32 * kSub)) {
    snprintf(msg, cap, "cand_cap must be a multiple of %d in [%d, 65536]", 32 * kSub, 32 * kSub);
    return RTS_E_INVALID;
  }
  if (!(c->lambda_v > 0 && c->lambda_f > 0 && c->alpha_rts > 0 && c->beta2 > 0 && c->beta_ratio > 0)) {
    snprintf(msg, cap, "time-step coefficients must be positive");
    return RTS_E_INVALID;
  }
  double nb = 1;
  for (int d = 0; d < 3; ++d) {
    double ext = c->domain_max[d] - c->domain_min[d];
    if (!(ext > 0)) { snprintf(msg, cap, "empty domain on axis %d", d); return RTS_E_INVALID; }
    nb *= ceil(ext / c->block_edge);
  }
  if (nb > 2.0e9) { snprintf(msg, cap, "too many blocks (%g)", nb); return RTS_E_INVALID; }
  return RTS_OK;
}

// What depends on the base step dtb: the step itself, the level thresholds
// and, for PCISPH, the pressure coefficient.  Level l steps 2^l base steps
// and takes beta of rank l + 1 (Section 3.1: beta_1 = infinity, beta_n =
// beta2 * ratio^(n-2)):
//   Eq. 3:  |v|^2 <= (alpha beta_{l+1} r / (2^l dt))^2
//   Eq. 2:  |a|^2 <= (lambda_f^2 r / (2^l dt)^2)^2
// PCISPH region n = l + 1 steps n base steps instead (Section 5).
void step_params(const rts_config &c, double mass, double dtb, DevParams &p) {
  const double rc = r_crit_of(c);
  p.dt_base = (float)dtb;
  for (int l = 0; l < kMaxLevels; ++l) {
    double dtl = c.solver == RTS_PCISPH ? dtb * (double)(l + 1) : ldexp(dtb, l);
    double bet = (l + 1 <= 1) ? INFINITY : c.beta2 * pow(c.beta_ratio, (double)(l + 1 - 2));
    double vl = isinf(bet) ? INFINITY : c.alpha_rts * bet * rc / dtl;
    double al = c.lambda_f * c.lambda_f * rc / (dtl * dtl);
    p.TV[l] = (float)(vl * vl);
    p.TA[l] = (float)(al * al);
  }
  if (c.solver == RTS_PCISPH) p.delta = (float)(c.delta > 0.0 ? c.delta : pci_delta(c, mass, dtb));
}

void derive(const rts_config &c, int64_t ncap, int64_t nwcap, DevParams &p, double &mass,
            double &B, double &dtb) {
  memset(&p, 0, sizeof(p));
  p.ncap = (int32_t)ncap;
  p.cand_cap = c.cand_cap;
  p.nbr_cap = c.nbr_cap;
  p.nbr_stride = (c.nbr_cap + 1 + 63) / 64 * 64 + 64;
  int64_t nb = 1;
  for (int d = 0; d < 3; ++d) {
    int32_t n = (int32_t)ceil((c.domain_max[d] - c.domain_min[d]) / c.block_edge);
    p.nc[d] = n < 1 ? 1 : n;
    nb *= p.nc[d];
    p.o[d] = (float)c.domain_min[d];
    p.dmax[d] = (float)c.domain_max[d];
    p.g[d] = (float)c.gravity[d];
  }
  (void)nwcap;
  p.nb = (int32_t)nb;
  p.act_cap = (int32_t)((nb + kActParts - 1) / kActParts);
  p.inv_e = (float)(1.0 / c.block_edge);
  p.r2f = (float)(c.support * c.support);
  p.h = (float)c.h;
  p.inv_h = (float)(1.0 / c.h);
  const double sigma = 1.0 / (M_PI * c.h * c.h * c.h);
  p.sigma = (float)sigma;
  mass = c.mass > 0.0 ? c.mass : c.rho0 / lattice_w_sum(c);
  p.mass = (float)mass;
  p.rho0 = (float)c.rho0;
  const double cc = c.rho0 / (mass * sigma) - 1.0;
  p.c_hi = (float)cc;
  p.c_lo = (float)(cc - (double)p.c_hi);
  const double cs = c.rho0 / (mass * sigma);
  p.cs_hi = (float)cs;
  p.cs_lo = (float)(cs - (double)p.cs_hi);
  p.kms = (float)(mass * sigma / c.rho0);
  B = c.B > 0.0 ? c.B : c.rho0 * c.c0 * c.c0 / c.gamma;
  p.B = (float)B;
  p.visc_num = (float)(2.0 * c.visc_alpha * c.h * c.c0);
  p.visc_eps_h2 = (float)(c.visc_eps * c.h * c.h);
  const double rc = r_crit_of(c);
  dtb = c.dt_base > 0.0 ? c.dt_base : c.lambda_v * rc / c.c0;   // Eq. 1
  p.dt_cfl = c.lambda_v * rc / c.c0;
  p.lf2r = c.lambda_f * c.lambda_f * rc;
  int lmax = c.n_levels - 1;
  if (c.level_cap < lmax) lmax = c.level_cap < 0 ? 0 : c.level_cap;
  if (c.mode != RTS_MODE_RTS) lmax = 0;
  p.lmax = lmax;
  p.mode = c.mode;
  p.serna_correct = c.serna_correct;
  p.clamp_p = c.clamp_p;
  p.phase_align = c.phase_align;
  p.solver = c.solver;
  p.support = (float)c.support;
  if (c.solver == RTS_PCISPH) {
    p.two_ring_levels = c.two_ring_levels > 0 ? c.two_ring_levels : 1;
    const double rl = c.r_list > 0.0 ? c.r_list : c.block_edge;
    p.r2l = (float)(rl * rl);
    p.eta_half = (float)(0.5 * c.eta);
    p.pci_nu = (float)(c.visc_alpha * c.h * c.c0 / c.rho0);
    p.w0m = (float)(mass * sigma);
  }
  step_params(c, mass, dtb, p);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Carves the workspace; with base == nullptr only the size is computed.
size_t carve(const DevParams &p, int64_t ncap, int64_t nwcap, char *base, DevPtrs *d) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char * {
    char *q = base ? base + off : nullptr;
    off += align256(bytes > 0 ? bytes : 1);
    return q;
  };
  const size_t n = (size_t)(ncap > 0 ? ncap : 1);
  const size_t nw = (size_t)(nwcap > 0 ? nwcap : 1);
  const size_t nb = (size_t)p.nb;
  const size_t ntiles = (nb + kScanTile - 1) / kScanTile;
  DevPtrs t;
  memset(&t, 0, sizeof(t));
  for (int b = 0; b < 2; ++b) {
    t.P[b] = (float4 *)take(n * 16);
    t.V[b] = (float4 *)take(n * 16);
    t.A[b] = (float4 *)take(n * 16);
    t.M[b] = (uint32_t *)take(n * 4);
    t.ID[b] = (uint32_t *)take(n * 4);
  }
  t.ANEW = (float4 *)take(n * 16);
  t.PRES = (float *)take(n * 4);
  t.KEY = (uint32_t *)take(n * 4);
  t.KEYOLD = (uint32_t *)take(n * 4);
  t.RANK = (uint32_t *)take(n * 4);
  t.TMP = (uint32_t *)take(n * 4);
  t.PERM = (uint32_t *)take(n * 4);
  t.NNB = (uint32_t *)take(n * 4);
  t.LIST = (uint16_t *)take(p.solver == RTS_PCISPH ? 4 : n * (size_t)p.nbr_stride * 2);
  t.COUNT = (uint32_t *)take(nb * 4);
  t.CELL_START = (uint32_t *)take((nb + 1) * 4);
  t.OCC = (uint32_t *)take(nb * 4);
  t.OCCR = (uint4 *)take(nb * 16);
  t.ACT = (uint32_t *)take((size_t)p.act_cap * kActBuckets * 4);
  t.ACTN = (uint32_t *)take((size_t)kActBuckets * kActnStride * 4);
  t.LRAW = (uint8_t *)take(nb);
  t.LVL = (uint8_t *)take(nb);
  t.BLKU = (uint4 *)take(nb * 16);
  t.BLKERR = (float *)take(nb * 4);
  t.BLKAMAX = (float *)take(nb * 4);
  t.PART = (StatPart *)take(sizeof(StatPart) * kStatBlocks);
  t.WP = (float4 *)take(nw * 16);
  t.WID = (uint32_t *)take(nw * 4);
  t.WCELL_START = (uint32_t *)take((nb + 1) * 4);
  t.WKEY = (uint32_t *)take(nw * 4);
  t.WRANK = (uint32_t *)take(nw * 4);
  t.WTMP = (uint32_t *)take(nw * 4);
  t.TILES = (unsigned long long *)take(ntiles * 8);
  t.TILES2 = (unsigned long long *)take(ntiles * 8);
  t.CTRL = (DevCtrl *)take(sizeof(DevCtrl));
  t.S = (DevScalars *)take(sizeof(DevScalars));
  const bool pci = p.solver == RTS_PCISPH;
  const size_t np = pci ? n : 1, nbp = pci ? nb : 1;
  t.XS = (float4 *)take(np * 16);
  t.PV = (float4 *)take(np * 16);
  t.FVG = (float4 *)take(np * 16);
  t.FP = (float4 *)take(np * 16);
  t.PQ = (float *)take(np * 4);
  t.SE = (uint8_t *)take(np);
  // lists in quads of entries: capacity rounded up to a multiple of four
  t.NBRL = (uint32_t *)take(np * (size_t)(pci ? (p.nbr_cap + 3) / 4 * 4 : 1) * 4);
  t.OB = (uint8_t *)take(nbp);
  t.NEARSE = (uint8_t *)take(nbp);
  t.DIL1 = (uint8_t *)take(nbp);
  t.DIL2 = (uint8_t *)take(nbp);
  t.DILT = (uint8_t *)take(nbp);
  t.DILATED = (uint8_t *)take(nbp);
  t.DEM = (uint32_t *)take(nbp * 4);
  t.PPART = (PciPart *)take(sizeof(PciPart) * kPciStatBlocks);
  t.PCI = (DevPci *)take(sizeof(DevPci));
  t.SCN_OFF = (uint32_t *)take((size_t)(kMaxScenes + 1) * 4);
  t.SCN_STAT = (SceneStat *)take(sizeof(SceneStat) * (size_t)kMaxScenes);
  if (d) *d = t;
  return off;
}

void destroy_graphs(rts_ctx *c) {
  for (int k = 0; k < 2; ++k) {
    if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
    if (c->graph[k]) (void)hipGraphDestroy(c->graph[k]);
    c->gexec[k] = nullptr;
    c->graph[k] = nullptr;
  }
  c->graph_ok = false;
}

bool fixed_step(const rts_ctx *c) { return c->prm.mode != RTS_MODE_GLOBAL_ADAPTIVE; }

// The kernels of one base step, reading buffer `cur` and leaving the state in
// buffer cur ^ 1.  With a fixed base step the binning of buffer `cur` was
// done by the previous step's closing kernel (or by rts_advance's prologue)
// and this step's closing kernel bins buffer cur ^ 1.
void enqueue_step(rts_ctx *c, int cur, hipStream_t st) {
  const DevParams &p = c->prm;
  const DevPtrs &d = c->d;
  const int nx = cur ^ 1;
  if (!fixed_step(c)) launch_key_hist(p, d, cur, st);
  launch_scan(p, d, d.CELL_START, true, st);
  launch_scatter(p, d, st);
  launch_cell_gather(p, d, cur, c->grid_wave, st);
  launch_rmin_flags(p, d, nx, 1, c->grid_wave, st);
  launch_search_density(p, d, nx, c->grid_search, c->search_threads, st);
  launch_force(p, d, nx, c->grid_force, c->force_lanes, st);
  if (fixed_step(c)) {
    launch_stats_correct_predict(p, d, nx, st);
  } else {
    // the step length comes from this step's statistics
    launch_step_stats(p, d, st);
    launch_correct_predict(p, d, nx, st);
  }
}

// Clears the block counts a closing kernel left for the next sort, before
// anything else sorts or the particles change.
rts_status unbin(rts_ctx *c) {
  if (!c->binned) return RTS_OK;
  c->binned = false;
  launch_fill(c->d.COUNT, 0, (size_t)c->prm.nb * 4, c->stream);
  HIP_OK(c, hipGetLastError());
  return RTS_OK;
}

rts_status build_graphs(rts_ctx *c) {
  destroy_graphs(c);
  if (!c->cap_stream)
    HIP_OK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  for (int k = 0; k < 2; ++k) {
    HIP_OK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
    enqueue_step(c, k, c->cap_stream);
    HIP_OK(c, hipStreamEndCapture(c->cap_stream, &c->graph[k]));
    HIP_OK(c, hipGraphInstantiate(&c->gexec[k], c->graph[k], nullptr, nullptr, 0));
  }
  c->graph_ok = true;
  return RTS_OK;
}

// Figure "iterations" of Section 5 (the image is not part of the text we
// work from): a schedule meeting every constraint the text states.  Bit l is
// region l + 1; rows 1-3 of minor-step columns (a)-(d).
uint32_t pci_turn(int col, int row) {
  static const uint32_t table[3][4] = {{0xF, 0xF, 0xF, 0xF}, {0xF, 0x1, 0x3, 0x1},
                                       {0x1, 0x1, 0x1, 0x1}};
  if (row < 1 || row > 3 || col < 0 || col > 3) return 0u;
  return table[row - 1][col];
}

// Algorithm 2, set-up of a major step: sort into the grid, regions from
// Eq. 2-3, dilation of regions 1 and 2, R_min, observed blocks, flags.
rts_status pci_major_begin(rts_ctx *c) {
  const DevParams &p = c->prm;
  const DevPtrs &d = c->d;
  hipStream_t st = c->stream;
  const int cur = c->cur, nx = cur ^ 1;
  // what a roll-back of this major step restores besides the particles
  c->snap_time = c->pci_time;
  c->snap_steps = c->pci_steps;
  c->snap_major_len = c->pci_major_len;
  c->snap_clean = c->pci_clean;
  c->pci_peak = 0;
  launch_key_hist(p, d, cur, st);
  launch_scan(p, d, d.CELL_START, true, st);
  launch_scatter(p, d, st);
  launch_cell_gather(p, d, cur, c->grid_wave, st);
  launch_pci_dilate(p, d, d.LRAW, d.DILT, 0, c->cfg.expand_layers, st);
  launch_pci_dilate(p, d, d.DILT, d.DILATED, 1, c->cfg.expand_layers, st);
  launch_rmin_flags(p, d, nx, 0, c->grid_wave, st, d.DILATED);
  launch_pci_observed(p, d, st);
  launch_pci_major_flags(p, d, nx, c->pci_major_len, st);
  HIP_OK(c, hipGetLastError());
  c->cur = nx;
  c->pci_ready = true;
  c->pci_excess = 0;
  return RTS_OK;
}

rts_status pci_read(rts_ctx *c, DevPci *h) {
  HIP_OK(c, hipMemcpyAsync(h, c->d.PCI, sizeof(DevPci), hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  return RTS_OK;
}

double pci_dt_lo(const rts_config &c) { return c.pci_dt_min > 0 ? c.pci_dt_min : 0.25 * c.dt_base; }

// Adaptive base step: the next major step's base step from the effort of
// the one just ended and the fastest particle after it (squared maxima, in
// float).  Eq. 3 takes beta_2: beta_1 = infinity bounds nothing.
double pci_next_dt(const rts_config &c, double dt, int peak, int excess, float v2max,
                   float a2max) {
  const int grow_at = c.pci_grow_iters > 0 ? c.pci_grow_iters : c.it_min;
  const int shrink_at = c.pci_shrink_iters > 0 ? c.pci_shrink_iters : c.it_min;
  const double hi = c.pci_dt_max > 0 ? c.pci_dt_max : 4.0 * c.dt_base;
  double next = (excess || peak > shrink_at) ? dt * c.pci_shrink
                                             : (peak <= grow_at ? dt * c.pci_grow : dt);
  next = fmin(next, hi);
  const double r = r_crit_of(c);
  if (v2max > 0.0f) next = fmin(next, c.alpha_rts * c.beta2 * r / sqrt((double)v2max));
  if (a2max > 0.0f) next = fmin(next, c.lambda_f * sqrt(r / sqrt((double)a2max)));
  return fmax(next, pci_dt_lo(c));
}

void pci_set_step(rts_ctx *c, double dt) {
  c->dt_base = dt;
  step_params(c->cfg, c->mass, dt, c->prm);
}

// One minor step of Algorithm 2 with the density correction of Algorithm 3.
rts_status pci_minor_step(rts_ctx *c) {
  const bool standard = c->cfg.mode != RTS_MODE_RTS;
  const bool adapt = !standard && c->cfg.pci_adapt_dt;
  if (standard) c->pci_major_len = 1;
  if (!c->pci_ready) {
    rts_status s = pci_major_begin(c);
    if (s) return s;
  }
  const DevParams &p = c->prm;
  const DevPtrs &d = c->d;
  hipStream_t st = c->stream;
  const int cur = c->cur, col = c->pci_minor_in_major;
  launch_pci_lists(p, d, cur, st);
  launch_pci_reset(p, d, st);
  HIP_OK(c, hipGetLastError());
  int iter = 1, row = 1, min_iter = c->cfg.it_min, global = 1, local_iters = 0;
  bool local_off = false;   // the minor step's one local phase has ended
  int global_iters = 0, resets = 0, reverts = 0;
  double errmax = INFINITY, avg = 0.0;
  const double eta = c->cfg.eta;
  DevPci h;
  while ((iter <= min_iter || errmax >= eta) && iter <= c->cfg.it_max) {
    const uint32_t turn = standard ? 0xFu : (global ? pci_turn(col, row) : 0u);
    launch_pci_predict(p, d, cur, st);
    launch_pci_density(p, d, cur, turn, st);
    launch_pci_mark_se(p, d, st);
    launch_pci_force(p, d, cur, turn, st);
    if (global) ++global_iters;
    ++iter;
    ++row;
    // the reductions decide only whether to stop (after min_iter iterations)
    // and the extra iterations (after the three scheduled rows): before both,
    // the loop goes on without waiting for the device
    const bool need = iter > min_iter || iter > 3;
    if (iter == 2 || need) launch_pci_errstats(p, d, cur, iter == 2 ? 1 : 0, st);
    HIP_OK(c, hipGetLastError());
    if (!need) continue;
    rts_status s = pci_read(c, &h);
    if (s) return s;
    errmax = (double)h.errmax;
    avg = h.avg;
    // extra iterations after the three scheduled ones (Section 5)
    if (errmax >= eta && iter > 3) {
      ++min_iter;
      if (standard) continue;
      if (avg >= c->cfg.eta_T) {            // global error: restart the schedule
        if (!global) {
          launch_pci_pressure_copy(p, d, 0, st);
          ++reverts;
          local_off = true;
        }
        global = 1;
        row = 1;
        ++resets;
      } else if (local_off) {               // back to global for the rest of the step
        row = 1;
        ++resets;
      } else if (global) {                  // local corrections on S_e
        launch_pci_pressure_copy(p, d, 1, st);
        global = 0;
        local_iters = 0;
      } else if (++local_iters >= c->cfg.local_fail) {
        launch_pci_pressure_copy(p, d, 0, st);
        global = 1;
        local_off = true;
        row = 1;
        ++reverts;
      }
    }
  }
  launch_pci_integrate(p, d, cur, c->pci_major_len, st);
  if (!standard) launch_pci_demote(p, d, cur, c->pci_major_len, st);
  c->pci_last[0] = iter - 1;
  c->pci_last[1] = global_iters;
  c->pci_last[2] = resets;
  c->pci_last[3] = reverts;
  c->pci_errmax = errmax;
  c->pci_avg = avg;
  c->pci_iters_total += iter - 1;
  if (iter - 1 > c->pci_peak) c->pci_peak = iter - 1;
  const double dt = c->dt_base;
  c->dt_last = dt;
  c->pci_time += dt;
  c->pci_steps += 1;
  c->pci_minor_in_major += 1;
  int early = 0;
  if (!standard && global_iters > c->cfg.global_limit) {
    c->pci_excess = 1;
    if (c->pci_minor_in_major < c->pci_major_len) early = 1;
  }
  c->pci_last[4] = early;
  const bool ends = c->pci_minor_in_major >= c->pci_major_len || early;
  // region counts after the step, read by rts_sync; at the end of a major
  // step of the adaptive base step also the speed and acceleration maxima
  launch_pci_errstats(p, d, cur, 0, st, adapt && ends);
  HIP_OK(c, hipGetLastError());
  if (ends) {
    c->pci_minor_in_major = 0;
    c->pci_ready = false;
    if (adapt) {
      rts_status s = pci_read(c, &h);
      if (s) return s;
      pci_set_step(c, pci_next_dt(c->cfg, dt, c->pci_peak, c->pci_excess, h.v2max, h.a2max));
    }
    if (!standard) {
      const int shortened = c->cfg.n_minor < 2 ? c->cfg.n_minor : 2;
      if (c->pci_excess) {
        c->pci_major_len = shortened;
        c->pci_clean = 0;
      } else if (c->pci_major_len < c->cfg.n_minor && ++c->pci_clean >= c->cfg.short_majors) {
        c->pci_major_len = c->cfg.n_minor;
        c->pci_clean = 0;
      }
    }
  }
  // a correction that did not converge: back to the state the major step
  // started from (still in the sort's source buffers), restarted with half
  // the step
  const double lo = pci_dt_lo(c->cfg);
  if (adapt && errmax >= eta && dt > lo) {
    c->cur = cur ^ 1;
    c->pci_time = c->snap_time;
    c->pci_steps = c->snap_steps;
    c->pci_major_len = c->snap_major_len;
    c->pci_clean = c->snap_clean;
    c->pci_minor_in_major = 0;
    c->pci_ready = false;
    c->pci_rollbacks += 1;
    pci_set_step(c, fmax(0.5 * dt, lo));
  }
  return RTS_OK;
}

// Context set-up in a given workspace.  Launches kernels only: no device
// memory is allocated, and the stream for graph capture is created when
// the first graph is built.  static_dev >= 0 marks a context living in the
// library's static workspace of that device.
rts_status create_in(const rts_config *cfg, int64_t n_fluid_max, int64_t n_wall_max,
                     void *d_workspace, size_t bytes, void *hip_stream, int static_dev,
                     rts_ctx **out, int32_t n_scenes = 1, const int64_t *counts = nullptr) {
  if (!out) return RTS_E_INVALID;
  *out = nullptr;
  char msg[256];
  rts_status s = validate(cfg, msg, sizeof(msg));
  if (s) return s;
  if (!d_workspace || ((uintptr_t)d_workspace & 255u) || n_fluid_max < 0 || n_wall_max < 0 ||
      n_fluid_max > 0x7FFFFFFF || n_wall_max > 0x7FFFFFFF)
    return RTS_E_INVALID;
  rts_ctx *c = new (std::nothrow) rts_ctx();
  if (!c) return RTS_E_DEVICE;
  c->cfg = *cfg;
  c->ncap = n_fluid_max;
  c->nwcap = n_wall_max;
  c->static_dev = static_dev;
  c->batched = counts != nullptr;
  c->n_scenes = n_scenes;
  c->scene_off = new (std::nothrow) uint32_t[(size_t)n_scenes + 1];
  c->scene_fill = new (std::nothrow) int64_t[(size_t)n_scenes];
  if (!c->scene_off || !c->scene_fill) {
    delete[] c->scene_off;
    delete[] c->scene_fill;
    delete c;
    return RTS_E_DEVICE;
  }
  c->scene_off[0] = 0;
  for (int32_t s = 0; s < n_scenes; ++s) {
    c->scene_off[s + 1] = c->scene_off[s] + (uint32_t)(counts ? counts[s] : 0);
    c->scene_fill[s] = 0;
  }
  derive(*cfg, n_fluid_max, n_wall_max, c->prm, c->mass, c->B, c->dt_base);
  c->prm.n_scenes = n_scenes;
  size_t need = carve(c->prm, n_fluid_max, n_wall_max, nullptr, nullptr);
  if (bytes < need) {
    delete[] c->scene_off;
    delete[] c->scene_fill;
    delete c;
    return RTS_E_CAPACITY;
  }
  carve(c->prm, n_fluid_max, n_wall_max, (char *)d_workspace, &c->d);
  c->ws = (char *)d_workspace;
  c->ws_used = need;
  c->stream = (hipStream_t)hip_stream;
  c->cur = 0;
  int dev = 0;
  (void)hipGetDevice(&dev);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    delete[] c->scene_off;
    delete[] c->scene_fill;
    delete c;
    return RTS_E_DEVICE;
  }
  const int cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  // persistent grids: enough workgroups to fill every CU, each striding over
  // the occupied blocks or taking active blocks by ticket (search and force:
  // two 512-thread workgroups per CU are resident, limited by registers)
  c->grid_wave = cus * 8;
  c->grid_search = cus * 3;
  c->grid_force = cus * 2;
  c->search_threads = 512;
  c->force_lanes = 8;
  // counts must start at zero; everything else is written before it is read
  hipStream_t st = c->stream;
  const size_t tiles = ((size_t)c->prm.nb + kScanTile - 1) / kScanTile * 8;
  launch_fill(c->d.COUNT, 0, (size_t)c->prm.nb * 4, st);
  launch_fill(c->d.TILES, 0, tiles, st);
  launch_fill(c->d.TILES2, 0, tiles, st);
  launch_fill(c->d.NNB, 0, (size_t)(n_fluid_max > 0 ? n_fluid_max : 1) * 4, st);
  launch_fill(c->d.WCELL_START, 0, ((size_t)c->prm.nb + 1) * 4, st);
  launch_fill(c->d.CTRL, 0, sizeof(DevCtrl), st);
  if (cfg->solver == RTS_PCISPH) {
    launch_fill(c->d.DEM, 0xFF, (size_t)c->prm.nb * 4, st);
    launch_fill(c->d.PCI, 0, sizeof(DevPci), st);
    launch_fill(c->d.OB, 0, (size_t)c->prm.nb, st);
  }
  c->pci_major_len = cfg->mode == RTS_MODE_RTS ? cfg->n_minor : 1;
  launch_reset_scalars(c->d.S, st);
  if (hipGetLastError() != hipSuccess) {
    delete[] c->scene_off;
    delete[] c->scene_fill;
    delete c;
    return RTS_E_DEVICE;
  }
  *out = c;
  return RTS_OK;
}

// A new run of n particles: counters, buffer parity and scene offsets reset
// (the particles themselves are written by the caller of this helper).
rts_status reset_run(rts_ctx *c, int32_t n) {
  rts_status u = unbin(c);
  if (u) return u;
  c->prm.n = n;
  c->cur = 0;
  c->pci_major_len = c->cfg.mode == RTS_MODE_RTS ? c->cfg.n_minor : 1;
  c->pci_minor_in_major = 0;
  c->pci_clean = 0;
  c->pci_excess = 0;
  c->pci_ready = false;
  c->pci_steps = 0;
  c->pci_iters_total = 0;
  c->pci_time = 0.0;
  c->pci_rollbacks = 0;
  if (c->cfg.solver == RTS_PCISPH) pci_set_step(c, c->cfg.dt_base);
  if (!c->batched) c->scene_off[1] = (uint32_t)n;
  for (int32_t s = 0; s < c->n_scenes; ++s) c->scene_fill[s] = 0;
  HIP_OK(c, hipMemcpyAsync(c->d.SCN_OFF, c->scene_off, ((size_t)c->n_scenes + 1) * 4,
                           hipMemcpyHostToDevice, c->stream));
  launch_reset_scalars(c->d.S, c->stream);
  HIP_OK(c, hipGetLastError());
  destroy_graphs(c);
  c->fresh = true;
  return RTS_OK;
}

bool scenes_complete(const rts_ctx *c) {
  for (int32_t s = 0; s < c->n_scenes; ++s)
    if (c->scene_fill[s] < (int64_t)(c->scene_off[s + 1] - c->scene_off[s])) return false;
  return true;
}

// Host side of a PCISPH run (the correction loop is driven from here),
// saved next to the workspace by rts_save_state.
struct PciHostState {
  int32_t n, nw, cur, major_len, minor_in_major, clean, excess, ready, peak, rollbacks;
  int32_t snap_major_len, snap_clean, last[6], hist[4];
  int64_t steps, iters_total, snap_steps;
  double time, dt_base, dt_last, snap_time, errmax, avg;
};
static_assert(sizeof(PciHostState) <= 192, "PCISPH host state fits its header slot");
constexpr int64_t kMagicWcsph = 0x5254535354415445LL;   // WCSPH particle state
constexpr int64_t kMagicPcisph = 0x5254535043495354LL;  // PCISPH workspace image
constexpr size_t kPciHeader = 256;                      // 64-byte header + host state

void pci_host_save(const rts_ctx *c, PciHostState &h) {
  memset(&h, 0, sizeof(h));
  h.n = c->prm.n; h.nw = c->prm.nw; h.cur = c->cur;
  h.major_len = c->pci_major_len; h.minor_in_major = c->pci_minor_in_major;
  h.clean = c->pci_clean; h.excess = c->pci_excess; h.ready = c->pci_ready ? 1 : 0;
  h.peak = c->pci_peak; h.rollbacks = c->pci_rollbacks;
  h.snap_major_len = c->snap_major_len; h.snap_clean = c->snap_clean;
  for (int k = 0; k < 6; ++k) h.last[k] = c->pci_last[k];
  for (int k = 0; k < 4; ++k) h.hist[k] = c->pci_hist[k];
  h.steps = c->pci_steps; h.iters_total = c->pci_iters_total; h.snap_steps = c->snap_steps;
  h.time = c->pci_time; h.dt_base = c->dt_base; h.dt_last = c->dt_last;
  h.snap_time = c->snap_time; h.errmax = c->pci_errmax; h.avg = c->pci_avg;
}

void pci_host_load(rts_ctx *c, const PciHostState &h) {
  c->prm.n = h.n; c->prm.nw = h.nw; c->cur = h.cur;
  c->pci_major_len = h.major_len; c->pci_minor_in_major = h.minor_in_major;
  c->pci_clean = h.clean; c->pci_excess = h.excess; c->pci_ready = h.ready != 0;
  c->pci_peak = h.peak; c->pci_rollbacks = h.rollbacks;
  c->snap_major_len = h.snap_major_len; c->snap_clean = h.snap_clean;
  for (int k = 0; k < 6; ++k) c->pci_last[k] = h.last[k];
  for (int k = 0; k < 4; ++k) c->pci_hist[k] = h.hist[k];
  c->pci_steps = h.steps; c->pci_iters_total = h.iters_total; c->snap_steps = h.snap_steps;
  c->pci_time = h.time; c->dt_last = h.dt_last; c->snap_time = h.snap_time;
  c->pci_errmax = h.errmax; c->pci_avg = h.avg;
  pci_set_step(c, h.dt_base);
}

}  // namespace

extern "C" {

void rts_default_config(rts_config *c) {
  memset(c, 0, sizeof(*c));
  c->solver = RTS_WCSPH;
  c->mode = RTS_MODE_RTS;
  c->n_levels = 4;
  c->level_cap = 3;
  c->clamp_p = 1;
  c->serna_correct = 1;
  c->cand_cap = 4096;
  c->use_graph = 1;
  c->spacing = 0.01;
  c->h = 0.02;
  c->support = 0.04;
  c->block_edge = 0.04;
  c->r_crit = 0.02;
  c->rho0 = 1000.0;
  c->mass = 0.0;
  c->c0 = 88.58893836;  // 20 sqrt(2 g H) for a 1 m column
  c->gamma = 7.0;
  c->B = 0.0;
  c->visc_alpha = 0.05;
  c->visc_eps = 0.01;
  c->gravity[1] = -9.81;
  for (int d = 0; d < 3; ++d) { c->domain_min[d] = -0.04; c->domain_max[d] = 1.04; }
  c->domain_max[0] = 2.04;
  c->dt_base = 0.0;
  c->lambda_v = 0.4;
  c->lambda_f = 0.25;
  c->alpha_rts = 0.4;
  c->beta2 = 0.4;
  c->beta_ratio = 0.2;
  c->n_minor = 4;
  c->it_min = 3;
  c->it_max = 50;
  c->expand_layers = 4;
  c->local_fail = 3;
  c->global_limit = 6;
  c->short_majors = 10;
  c->nbr_cap = 512;
  c->two_ring_levels = 1;
  c->eta = 0.01;
  c->eta_T = 0.0025;
  c->delta = 0.0;
  c->r_list = 0.0;
  c->pci_adapt_dt = 0;
  c->pci_grow_iters = 0;
  c->pci_shrink_iters = 0;
  c->pci_dt_min = 0.0;
  c->pci_dt_max = 0.0;
  c->pci_grow = 1.02;
  c->pci_shrink = 0.95;
  c->phase_align = 1;
}

const char *rts_status_string(rts_status s) {
  switch (s) {
    case RTS_OK: return "ok";
    case RTS_E_INVALID: return "invalid argument";
    case RTS_E_CAPACITY: return "capacity exceeded";
    case RTS_E_DEVICE: return "device error";
    case RTS_E_NUMERICAL: return "numerical failure";
    case RTS_E_STATE: return "invalid state";
    case RTS_E_UNSUPPORTED: return "unsupported";
  }
  return "unknown";
}

const char *rts_last_error(const rts_ctx *c) { return c ? c->err : "no context"; }

rts_status rts_workspace_size(const rts_config *cfg, int64_t n_fluid_max, int64_t n_wall_max,
                              size_t *bytes) {
  char msg[256];
  rts_status s = validate(cfg, msg, sizeof(msg));
  if (s) return s;
  if (!bytes || n_fluid_max < 0 || n_wall_max < 0 || n_fluid_max > 0x7FFFFFFF ||
      n_wall_max > 0x7FFFFFFF)
    return RTS_E_INVALID;
  DevParams p;
  double m, B, dt;
  derive(*cfg, n_fluid_max, n_wall_max, p, m, B, dt);
  *bytes = carve(p, n_fluid_max, n_wall_max, nullptr, nullptr);
  return RTS_OK;
}

rts_status rts_create(const rts_config *cfg, int64_t n_fluid_max, int64_t n_wall_max,
                      void *d_workspace, size_t bytes, void *hip_stream, rts_ctx **out) {
  return create_in(cfg, n_fluid_max, n_wall_max, d_workspace, bytes, hip_stream, -1, out);
}

rts_status rts_create_static(const rts_config *cfg, int64_t n_fluid_max, int64_t n_wall_max,
                             void *hip_stream, rts_ctx **out) {
  if (!out) return RTS_E_INVALID;
  *out = nullptr;
  size_t need = 0;
  rts_status s = rts_workspace_size(cfg, n_fluid_max, n_wall_max, &need);
  if (s) return s;
  if (need > (size_t)RTS_STATIC_WORKSPACE_BYTES) return RTS_E_CAPACITY;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return RTS_E_DEVICE;
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (!g_static_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return RTS_E_DEVICE;
    g_static_ptr[dev] = p;
  }
  if (g_static_busy[dev]) return RTS_E_STATE;
  s = create_in(cfg, n_fluid_max, n_wall_max, g_static_ptr[dev],
                (size_t)RTS_STATIC_WORKSPACE_BYTES, hip_stream, dev, out);
  if (s == RTS_OK) g_static_busy[dev] = true;
  return s;
}

rts_status rts_create_batch(const rts_config *cfg, int32_t n_scenes, const int64_t *h_n_per_scene,
                            int64_t n_wall_max, void *d_workspace, size_t bytes,
                            void *hip_stream, rts_ctx **out) {
  if (!out) return RTS_E_INVALID;
  *out = nullptr;
  if (!cfg || !h_n_per_scene || n_scenes < 1 || n_scenes > RTS_MAX_SCENES) return RTS_E_INVALID;
  if (cfg->solver != RTS_WCSPH) return RTS_E_UNSUPPORTED;
  int64_t total = 0;
  for (int32_t s = 0; s < n_scenes; ++s) {
    if (h_n_per_scene[s] < 0) return RTS_E_INVALID;
    total += h_n_per_scene[s];
  }
  if (total > 0x7FFFFFFF) return RTS_E_INVALID;
  return create_in(cfg, total, n_wall_max, d_workspace, bytes, hip_stream, -1, out, n_scenes,
                   h_n_per_scene);
}

void rts_destroy(rts_ctx *c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  destroy_graphs(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->static_dev >= 0) {
    std::lock_guard<std::mutex> lock(g_static_mu);
    g_static_busy[c->static_dev] = false;
  }
  delete[] c->scene_off;
  delete[] c->scene_fill;
  delete c;
}

rts_status rts_set_walls(rts_ctx *c, const float *d_pos, int64_t nw) {
  if (!c) return RTS_E_INVALID;
  if (nw < 0 || nw > c->nwcap) return fail(c, RTS_E_CAPACITY, "nw %lld exceeds capacity %lld", (long long)nw, (long long)c->nwcap);
  if (nw > 0 && !d_pos) return fail(c, RTS_E_INVALID, "wall positions are NULL");
  rts_status u = unbin(c);  // the wall sort counts in the same array
  if (u) return u;
  c->prm.nw = (int32_t)nw;
  launch_wall_sort(c->prm, c->d, d_pos, c->stream);
  HIP_OK(c, hipGetLastError());
  destroy_graphs(c);
  return RTS_OK;
}

rts_status rts_set_state(rts_ctx *c, const float *d_pos, const float *d_vel, int64_t n) {
  if (!c) return RTS_E_INVALID;
  if (n < 0 || n > c->ncap) return fail(c, RTS_E_CAPACITY, "n %lld exceeds capacity %lld", (long long)n, (long long)c->ncap);
  if (n > 0 && !d_pos) return fail(c, RTS_E_INVALID, "positions are NULL");
  if (c->batched && n != (int64_t)c->scene_off[c->n_scenes])
    return fail(c, RTS_E_INVALID, "a batch of %d scenes holds %u particles, not %lld",
                c->n_scenes, c->scene_off[c->n_scenes], (long long)n);
  rts_status u = reset_run(c, (int32_t)n);
  if (u) return u;
  for (int32_t s = 0; s < c->n_scenes; ++s)
    c->scene_fill[s] = (int64_t)(c->scene_off[s + 1] - c->scene_off[s]);
  launch_set_state(c->prm, c->d, 0, d_pos, d_vel, c->stream);
  HIP_OK(c, hipGetLastError());
  c->has_state = true;
  c->poisoned = false;
  return RTS_OK;
}

rts_status rts_add_velocity(rts_ctx *c, const float *d_dv, int64_t n) {
  if (!c) return RTS_E_INVALID;
  if (!c->has_state) return fail(c, RTS_E_STATE, "no state");
  if (n != (int64_t)c->prm.n)
    return fail(c, RTS_E_INVALID, "n %lld differs from the particle count %d", (long long)n,
                c->prm.n);
  if (n > 0 && !d_dv) return fail(c, RTS_E_INVALID, "velocity changes are NULL");
  launch_add_velocity(c->prm, c->d, c->cur, d_dv, c->stream);
  HIP_OK(c, hipGetLastError());
  return RTS_OK;
}

rts_status rts_init_dam_break(rts_ctx *c, int32_t scene, int64_t first, const int32_t *h_counts,
                              const double *h_corner, double spacing, double jitter,
                              uint64_t seed, uint64_t first_draw) {
  if (!c) return RTS_E_INVALID;
  if (!c->batched)
    return fail(c, RTS_E_STATE, "scene sizes are fixed by rts_create_batch; this context "
                "takes its particles from rts_set_state");
  if (scene < 0 || scene >= c->n_scenes || !h_counts || !h_corner || first < 0)
    return fail(c, RTS_E_INVALID, "bad scene %d or column arguments", scene);
  int64_t cnt = 1;
  for (int a = 0; a < 3; ++a) {
    if (h_counts[a] < 0) return fail(c, RTS_E_INVALID, "negative lattice count");
    cnt *= h_counts[a];
  }
  const int64_t n_s = (int64_t)(c->scene_off[scene + 1] - c->scene_off[scene]);
  if (first + cnt > n_s)
    return fail(c, RTS_E_INVALID, "column of %lld particles from %lld exceeds scene %d's %lld",
                (long long)cnt, (long long)first, scene, (long long)n_s);
  if (!(spacing > 0.0) || !(jitter >= 0.0))
    return fail(c, RTS_E_INVALID, "spacing must be positive and jitter non-negative");
  if (!c->fresh) {
    // the first column after anything that sorted starts a new run of every scene
    rts_status u = reset_run(c, (int32_t)c->scene_off[c->n_scenes]);
    if (u) return u;
    c->has_state = false;
  }
  LatticeSpec L;
  memset(&L, 0, sizeof(L));
  for (int a = 0; a < 3; ++a) {
    L.counts[a] = h_counts[a];
    L.corner[a] = h_corner[a];
  }
  L.spacing = spacing;
  L.jitter = jitter;
  L.seed = seed;
  L.first_draw = first_draw;
  launch_init_lattice(c->prm, c->d, c->scene_off[scene] + (uint32_t)first, (uint32_t)cnt, L,
                      c->stream);
  HIP_OK(c, hipGetLastError());
  c->scene_fill[scene] += cnt;
  if (scenes_complete(c)) {
    c->has_state = true;
    c->poisoned = false;
  }
  return RTS_OK;
}

rts_status rts_get_scene_stats(rts_ctx *c, rts_scene_stats *h_out, int32_t n_scenes) {
  if (!c || !h_out) return RTS_E_INVALID;
  if (n_scenes != c->n_scenes)
    return fail(c, RTS_E_INVALID, "the context holds %d scenes", c->n_scenes);
  if (!c->has_state) return fail(c, RTS_E_STATE, "no state");
  launch_scene_stats(c->prm, c->d, c->cur, c->stream);
  HIP_OK(c, hipGetLastError());
  SceneStat *tmp = new (std::nothrow) SceneStat[(size_t)n_scenes];
  if (!tmp) return fail(c, RTS_E_DEVICE, "host memory");
  hipError_t e = hipMemcpyAsync(tmp, c->d.SCN_STAT, sizeof(SceneStat) * (size_t)n_scenes,
                                hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    delete[] tmp;
    return fail(c, RTS_E_DEVICE, "copy of the scene counters failed: %s", hipGetErrorString(e));
  }
  for (int32_t s = 0; s < n_scenes; ++s) {
    rts_scene_stats &o = h_out[s];
    memset(&o, 0, sizeof(o));
    o.first = c->scene_off[s];
    o.n = (int64_t)(c->scene_off[s + 1] - c->scene_off[s]);
    o.active_last = tmp[s].act;
    o.inter_last = (int64_t)tmp[s].inter;
    float err;
    memcpy(&err, &tmp[s].err_bits, 4);
    o.err_max_last = err;
    for (int l = 0; l < RTS_MAX_LEVELS; ++l) o.level_hist[l] = tmp[s].hist[l];
  }
  delete[] tmp;
  return RTS_OK;
}

rts_status rts_get_scene_state(rts_ctx *c, int32_t scene, float *d_pos, float *d_vel,
                               float *d_acc, float *d_rho, float *d_p, uint8_t *d_level) {
  if (!c) return RTS_E_INVALID;
  if (scene < 0 || scene >= c->n_scenes) return fail(c, RTS_E_INVALID, "bad scene %d", scene);
  if (!c->has_state) return fail(c, RTS_E_STATE, "no state");
  const uint32_t lo = c->scene_off[scene], cnt = c->scene_off[scene + 1] - lo;
  launch_get_range(c->prm, c->d, c->cur, lo, cnt, d_pos, d_vel, d_acc, d_rho, d_p, d_level,
                   c->stream);
  HIP_OK(c, hipGetLastError());
  return RTS_OK;
}

rts_status rts_assign_levels(rts_ctx *c, int32_t *h_hist) {
  if (!c) return RTS_E_INVALID;
  if (!c->has_state) return fail(c, RTS_E_STATE, "no state");
  c->fresh = false;
  const DevParams &p = c->prm;
  if (c->cfg.solver == RTS_PCISPH) {
    if (c->cfg.mode != RTS_MODE_RTS) c->pci_major_len = 1;
    rts_status s = pci_major_begin(c);
    if (s) return s;
    c->pci_minor_in_major = 0;
  } else {
    rts_status u = unbin(c);
    if (u) return u;
    const int cur = c->cur;
    launch_key_hist(p, c->d, cur, c->stream);
    launch_scan(p, c->d, c->d.CELL_START, true, c->stream);
    launch_scatter(p, c->d, c->stream);
    launch_cell_gather(p, c->d, cur, c->grid_wave, c->stream);
    launch_rmin_flags(p, c->d, cur ^ 1, 0, c->grid_wave, c->stream);
    HIP_OK(c, hipGetLastError());
    c->cur = cur ^ 1;
  }
  if (h_hist) {
    uint8_t *lv = (uint8_t *)malloc((size_t)p.nb);
    if (!lv) return RTS_E_DEVICE;
    hipError_t e = hipMemcpyAsync(lv, c->d.LVL, (size_t)p.nb, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
      free(lv);
      return fail(c, RTS_E_DEVICE, "copy of block levels failed: %s", hipGetErrorString(e));
    }
    for (int l = 0; l < c->cfg.n_levels; ++l) h_hist[l] = 0;
    for (int64_t b = 0; b < p.nb; ++b)
      if (lv[b] != kEmpty && lv[b] < c->cfg.n_levels) h_hist[lv[b]]++;
    free(lv);
  } else {
    HIP_OK(c, hipStreamSynchronize(c->stream));
  }
  return RTS_OK;
}

rts_status rts_advance(rts_ctx *c, int32_t n_steps) {
  if (!c || n_steps < 0) return RTS_E_INVALID;
  if (!c->has_state) return fail(c, RTS_E_STATE, "no state");
  if (c->poisoned) return fail(c, RTS_E_STATE, "state failed; set or load a state first");
  if (n_steps == 0) return RTS_OK;
  c->fresh = false;
  if (c->cfg.solver == RTS_PCISPH) {
    // accepted minor steps: a rolled-back major step takes pci_steps back
    const int64_t target = c->pci_steps + n_steps;
    while (c->pci_steps < target) {
      rts_status s = pci_minor_step(c);
      if (s) return s;
    }
    return RTS_OK;
  }
  if (c->cfg.use_graph && !c->graph_ok) {
    rts_status s = build_graphs(c);
    if (s) return s;
  }
  if (fixed_step(c) && !c->binned) {
    // the first step's binning, which later steps get from their predecessor
    launch_key_hist(c->prm, c->d, c->cur, c->stream);
    HIP_OK(c, hipGetLastError());
  }
  c->binned = fixed_step(c);
  for (int32_t k = 0; k < n_steps; ++k) {
    if (c->graph_ok) {
      HIP_OK(c, hipGraphLaunch(c->gexec[c->cur], c->stream));
    } else {
      enqueue_step(c, c->cur, c->stream);
      HIP_OK(c, hipGetLastError());
    }
    c->cur ^= 1;
  }
  return RTS_OK;
}

rts_status rts_profile_advance(rts_ctx *c, int32_t n_steps, double *h_ms) {
  if (c) c->fresh = false;
  if (!c || n_steps < 0 || !h_ms) return RTS_E_INVALID;
  if (c->cfg.solver == RTS_PCISPH)
    return fail(c, RTS_E_UNSUPPORTED, "per-kernel profiling covers the WCSPH step");
  if (!c->has_state) return fail(c, RTS_E_STATE, "no state");
  if (c->poisoned) return fail(c, RTS_E_STATE, "state failed; set or load a state first");
  // the kernels are launched one by one, binning included
  rts_status u = unbin(c);
  if (u) return u;
  hipEvent_t ev[RTS_PROF_COUNT + 1];
  for (int k = 0; k <= RTS_PROF_COUNT; ++k) HIP_OK(c, hipEventCreate(&ev[k]));
  rts_status st = RTS_OK;
  const DevParams &p = c->prm;
  const DevPtrs &d = c->d;
  for (int32_t s = 0; s < n_steps && st == RTS_OK; ++s) {
    const int cur = c->cur, nx = cur ^ 1;
    hipStream_t q = c->stream;
    (void)hipEventRecord(ev[0], q);
    launch_key_hist(p, d, cur, q);
    (void)hipEventRecord(ev[1], q);
    launch_scan(p, d, d.CELL_START, true, q);
    (void)hipEventRecord(ev[2], q);
    launch_scatter(p, d, q);
    (void)hipEventRecord(ev[3], q);
    launch_cell_gather(p, d, cur, c->grid_wave, q);
    (void)hipEventRecord(ev[4], q);
    launch_rmin_flags(p, d, nx, 1, c->grid_wave, q);
    (void)hipEventRecord(ev[5], q);
    launch_search_density(p, d, nx, c->grid_search, c->search_threads, q);
    (void)hipEventRecord(ev[6], q);
    launch_force(p, d, nx, c->grid_force, c->force_lanes, q);
    (void)hipEventRecord(ev[7], q);
    launch_step_stats(p, d, q);
    (void)hipEventRecord(ev[8], q);
    launch_correct_predict(p, d, nx, q);
    (void)hipEventRecord(ev[9], q);
    c->cur = nx;
    if (hipEventSynchronize(ev[RTS_PROF_COUNT]) != hipSuccess) {
      st = fail(c, RTS_E_DEVICE, "event synchronisation failed");
      break;
    }
    for (int k = 0; k < RTS_PROF_COUNT; ++k) {
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
      h_ms[k] += ms;
    }
  }
  for (int k = 0; k <= RTS_PROF_COUNT; ++k) (void)hipEventDestroy(ev[k]);
  return st;
}

rts_status rts_sync(rts_ctx *c, rts_stats *out) {
  if (!c) return RTS_E_INVALID;
  DevScalars S;
  HIP_OK(c, hipMemcpyAsync(&S, c->d.S, sizeof(S), hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  const int32_t bad = S.status ? S.bad_index : -1;
  if (out) {
    memset(out, 0, sizeof(*out));
    out->step = S.step;
    out->time = S.time;
    out->dt_last = S.dt_next;
    out->active_last = S.n_act;
    out->inter_last = (int64_t)S.inter_last;
    out->active_total = (int64_t)S.active_total;
    out->inter_total = (int64_t)S.inter_total;
    out->cand_total = (int64_t)S.cand_total;
    out->err_max_last = S.err_last;
    out->err_max_run = S.err_run;
    for (int l = 0; l < RTS_MAX_LEVELS; ++l) out->level_hist[l] = S.hist[l];
    out->nbr_max = (int32_t)S.nbr_max;
    out->status = (int32_t)S.status;
    out->bad_index = bad;
    if (c->cfg.solver == RTS_PCISPH) {
      DevPci h;
      HIP_OK(c, hipMemcpyAsync(&h, c->d.PCI, sizeof(h), hipMemcpyDeviceToHost, c->stream));
      HIP_OK(c, hipStreamSynchronize(c->stream));
      for (int k = 0; k < 4; ++k) c->pci_hist[k] = h.hist[k];
      c->pci_last[5] = h.ncomp_first;
      out->step = c->pci_steps;
      out->time = c->pci_time;
      out->dt_last = c->pci_steps > 0 ? c->dt_last : c->dt_base;
      out->pci_dt_next = c->dt_base;
      out->pci_rollbacks = c->pci_rollbacks;
      out->err_max_last = (float)c->pci_errmax;
      for (int l = 0; l < RTS_MAX_LEVELS; ++l) out->level_hist[l] = l < 4 ? c->pci_hist[l] : 0;
      out->pci_iters = c->pci_last[0];
      out->pci_global_iters = c->pci_last[1];
      out->pci_resets = c->pci_last[2];
      out->pci_reverts = c->pci_last[3];
      out->pci_early_end = c->pci_last[4];
      out->pci_lists = c->pci_last[5];
      out->pci_major_len = c->pci_major_len;
      out->pci_minor_in_major = c->pci_minor_in_major;
      out->pci_errmax = c->pci_errmax;
      out->pci_avg = c->pci_avg;
      out->pci_iters_total = c->pci_iters_total;
    }
  }
  if (S.status) {
    c->poisoned = true;
    return fail(c, (rts_status)S.status, "device reported %s (particle %d)",
                rts_status_string((rts_status)S.status), bad);
  }
  return RTS_OK;
}

rts_status rts_get_state(rts_ctx *c, float *d_pos, float *d_vel, float *d_acc, float *d_rho,
                         float *d_p, uint8_t *d_level) {
  if (!c) return RTS_E_INVALID;
  if (!c->has_state) return fail(c, RTS_E_STATE, "no state");
  launch_get_state(c->prm, c->d, c->cur, d_pos, d_vel, d_acc, d_rho, d_p, d_level, c->stream);
  HIP_OK(c, hipGetLastError());
  return RTS_OK;
}

rts_status rts_state_bytes(rts_ctx *c, size_t *bytes) {
  if (!c || !bytes) return RTS_E_INVALID;
  if (c->cfg.solver == RTS_PCISPH) {
    *bytes = kPciHeader + c->ws_used;
    return RTS_OK;
  }
  size_t n = (size_t)c->prm.n;
  *bytes = 64 + n * (16 * 3 + 4 * 3) + sizeof(DevScalars);
  return RTS_OK;
}

namespace {

// PCISPH: an image of the whole workspace (particles in both sort buffers,
// the major step's grid, regions and observed blocks, lists, non-pressure
// accelerations, errors, scan and control words) plus the host loop's
// counters, so that a restored run continues bit for bit at any minor step.
rts_status pci_save(rts_ctx *c, void *d_buf, size_t cap) {
  size_t need;
  rts_state_bytes(c, &need);
  if (cap < need) return fail(c, RTS_E_CAPACITY, "buffer holds %zu of %zu bytes", cap, need);
  char hdr[kPciHeader];
  memset(hdr, 0, sizeof(hdr));
  int64_t *h64 = (int64_t *)hdr;
  h64[0] = kMagicPcisph;
  h64[1] = c->ncap;
  h64[2] = c->nwcap;
  h64[3] = c->prm.nb;
  h64[4] = (int64_t)c->ws_used;
  h64[5] = c->cfg.mode;
  PciHostState hs;
  pci_host_save(c, hs);
  memcpy(hdr + 64, &hs, sizeof(hs));
  char *b = (char *)d_buf;
  HIP_OK(c, hipMemcpyAsync(b, hdr, kPciHeader, hipMemcpyHostToDevice, c->stream));
  HIP_OK(c, hipMemcpyAsync(b + kPciHeader, c->ws, c->ws_used, hipMemcpyDeviceToDevice,
                           c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));  // the header lives on this host stack
  return RTS_OK;
}

rts_status pci_load(rts_ctx *c, const void *d_buf, size_t len) {
  if (len < kPciHeader) return fail(c, RTS_E_INVALID, "buffer too short");
  char hdr[kPciHeader];
  HIP_OK(c, hipStreamSynchronize(c->stream));
  HIP_OK(c, hipMemcpy(hdr, d_buf, kPciHeader, hipMemcpyDeviceToHost));
  const int64_t *h64 = (const int64_t *)hdr;
  if (h64[0] != kMagicPcisph || h64[1] != c->ncap || h64[2] != c->nwcap ||
      h64[3] != c->prm.nb || h64[4] != (int64_t)c->ws_used || h64[5] != c->cfg.mode)
    return fail(c, RTS_E_INVALID, "buffer does not hold a PCISPH state for this context");
  if (len < kPciHeader + c->ws_used) return fail(c, RTS_E_INVALID, "buffer too short");
  PciHostState hs;
  memcpy(&hs, hdr + 64, sizeof(hs));
  HIP_OK(c, hipMemcpyAsync(c->ws, (const char *)d_buf + kPciHeader, c->ws_used,
                           hipMemcpyDeviceToDevice, c->stream));
  pci_host_load(c, hs);
  c->fresh = false;
  c->has_state = true;
  c->poisoned = false;
  return RTS_OK;
}

}  // namespace

rts_status rts_save_state(rts_ctx *c, void *d_buf, size_t cap) {
  if (!c || !d_buf) return RTS_E_INVALID;
  if (!c->has_state) return fail(c, RTS_E_STATE, "no state");
  if (c->cfg.solver == RTS_PCISPH) return pci_save(c, d_buf, cap);
  size_t need;
  rts_state_bytes(c, &need);
  if (cap < need) return fail(c, RTS_E_CAPACITY, "buffer holds %zu of %zu bytes", cap, need);
  size_t n = (size_t)c->prm.n;
  char *b = (char *)d_buf;
  int64_t hdr[8] = {kMagicWcsph, (int64_t)n, c->prm.nb, 0, 0, 0, 0, 0};
  HIP_OK(c, hipMemcpyAsync(b, hdr, 64, hipMemcpyHostToDevice, c->stream));
  size_t off = 64;
  const int k = c->cur;
  HIP_OK(c, hipMemcpyAsync(b + off, c->d.P[k], n * 16, hipMemcpyDeviceToDevice, c->stream)); off += n * 16;
  HIP_OK(c, hipMemcpyAsync(b + off, c->d.V[k], n * 16, hipMemcpyDeviceToDevice, c->stream)); off += n * 16;
  HIP_OK(c, hipMemcpyAsync(b + off, c->d.A[k], n * 16, hipMemcpyDeviceToDevice, c->stream)); off += n * 16;
  HIP_OK(c, hipMemcpyAsync(b + off, c->d.M[k], n * 4, hipMemcpyDeviceToDevice, c->stream)); off += n * 4;
  HIP_OK(c, hipMemcpyAsync(b + off, c->d.ID[k], n * 4, hipMemcpyDeviceToDevice, c->stream)); off += n * 4;
  HIP_OK(c, hipMemcpyAsync(b + off, c->d.PRES, n * 4, hipMemcpyDeviceToDevice, c->stream)); off += n * 4;
  HIP_OK(c, hipMemcpyAsync(b + off, c->d.S, sizeof(DevScalars), hipMemcpyDeviceToDevice, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));  // the header lives on this host stack
  return RTS_OK;
}

rts_status rts_load_state(rts_ctx *c, const void *d_buf, size_t len) {
  if (!c || !d_buf || len < 64) return RTS_E_INVALID;
  if (c->cfg.solver == RTS_PCISPH) return pci_load(c, d_buf, len);
  int64_t hdr[8];
  HIP_OK(c, hipMemcpy(hdr, d_buf, 64, hipMemcpyDeviceToHost));
  if (hdr[0] != kMagicWcsph || hdr[1] < 0 || hdr[1] > c->ncap || hdr[2] != c->prm.nb)
    return fail(c, RTS_E_INVALID, "buffer does not hold a state for this context");
  size_t n = (size_t)hdr[1];
  rts_status u = unbin(c);
  if (u) return u;
  const bool same_n = c->prm.n == (int32_t)n;
  c->prm.n = (int32_t)n;
  size_t need;
  rts_state_bytes(c, &need);
  if (len < need) return fail(c, RTS_E_INVALID, "buffer too short");
  const char *b = (const char *)d_buf;
  size_t off = 64;
  c->cur = 0;
  HIP_OK(c, hipMemcpyAsync(c->d.P[0], b + off, n * 16, hipMemcpyDeviceToDevice, c->stream)); off += n * 16;
  HIP_OK(c, hipMemcpyAsync(c->d.V[0], b + off, n * 16, hipMemcpyDeviceToDevice, c->stream)); off += n * 16;
  HIP_OK(c, hipMemcpyAsync(c->d.A[0], b + off, n * 16, hipMemcpyDeviceToDevice, c->stream)); off += n * 16;
  HIP_OK(c, hipMemcpyAsync(c->d.M[0], b + off, n * 4, hipMemcpyDeviceToDevice, c->stream)); off += n * 4;
  HIP_OK(c, hipMemcpyAsync(c->d.ID[0], b + off, n * 4, hipMemcpyDeviceToDevice, c->stream)); off += n * 4;
  HIP_OK(c, hipMemcpyAsync(c->d.PRES, b + off, n * 4, hipMemcpyDeviceToDevice, c->stream)); off += n * 4;
  HIP_OK(c, hipMemcpyAsync(c->d.S, b + off, sizeof(DevScalars), hipMemcpyDeviceToDevice, c->stream));
  // the graphs hold the particle count; buffers and both parities are fixed
  if (!same_n) destroy_graphs(c);
  c->fresh = false;
  c->has_state = true;
  c->poisoned = false;
  return RTS_OK;
}

rts_status rts_debug_get(rts_ctx *c, int32_t what, void *d_out, size_t cap, size_t *n_out) {
  if (!c || !d_out) return RTS_E_INVALID;
  const size_t n = (size_t)c->prm.n, nb = (size_t)c->prm.nb, nw = (size_t)c->prm.nw;
  const int k = c->cur, pk = c->cur ^ 1;
  const bool pci = c->cfg.solver == RTS_PCISPH;
  const void *src = nullptr;
  size_t count = 0, esz = 4;
  switch (what) {
    case RTS_DBG_POS: src = c->d.P[k]; count = n; esz = 16; break;
    case RTS_DBG_VEL: src = c->d.V[k]; count = n; esz = 16; break;
    case RTS_DBG_ACC: src = c->d.A[k]; count = n; esz = 16; break;
    case RTS_DBG_ACC_NEW: src = c->d.ANEW; count = n; esz = 16; break;
    case RTS_DBG_META: src = c->d.M[k]; count = n; break;
    case RTS_DBG_ID: src = c->d.ID[k]; count = n; break;
    case RTS_DBG_KEY: src = c->d.KEY; count = n; break;
    case RTS_DBG_PERM: src = c->d.PERM; count = n; break;
    case RTS_DBG_CELL_START: src = c->d.CELL_START; count = nb + 1; break;
    case RTS_DBG_BLK_LEVEL_RAW: src = c->d.LRAW; count = nb; esz = 1; break;
    case RTS_DBG_BLK_LEVEL: src = c->d.LVL; count = nb; esz = 1; break;
    case RTS_DBG_NNB: src = c->d.NNB; count = n; break;
    case RTS_DBG_NBR: {
      // canonical lists of the last step's active particles, then their counts
      count = n * ((size_t)RTS_DEBUG_NBR_ROW + 1);
      if (n_out) *n_out = count;
      if (count * 4 > cap) return fail(c, RTS_E_CAPACITY, "debug view needs %zu bytes", count * 4);
      uint32_t *o = (uint32_t *)d_out;
      launch_debug_lists(c->prm, c->d, k, o, o + n * (size_t)RTS_DEBUG_NBR_ROW, c->stream);
      HIP_OK(c, hipGetLastError());
      return RTS_OK;
    }
    case RTS_DBG_PRESSURE: src = c->d.PRES; count = n; break;
    case RTS_DBG_PRE_POS: src = c->d.P[pk]; count = n; esz = 16; break;
    case RTS_DBG_PRE_VEL: src = c->d.V[pk]; count = n; esz = 16; break;
    case RTS_DBG_PRE_ACC: src = c->d.A[pk]; count = n; esz = 16; break;
    case RTS_DBG_PRE_META: src = c->d.M[pk]; count = n; break;
    case RTS_DBG_PRE_ID: src = c->d.ID[pk]; count = n; break;
    case RTS_DBG_WALL_POS: src = c->d.WP; count = nw; esz = 16; break;
    case RTS_DBG_WALL_ID: src = c->d.WID; count = nw; break;
    case RTS_DBG_WALL_CELL_START: src = c->d.WCELL_START; count = nb + 1; break;
    case RTS_DBG_BLK_STATS: src = c->d.BLKU; count = nb; esz = 16; break;
    case RTS_DBG_PCI_XS: src = c->d.XS; count = pci ? n : 0; esz = 16; break;
    case RTS_DBG_PCI_PV: src = c->d.PV; count = pci ? n : 0; esz = 16; break;
    case RTS_DBG_PCI_FVG: src = c->d.FVG; count = pci ? n : 0; esz = 16; break;
    case RTS_DBG_PCI_FP: src = c->d.FP; count = pci ? n : 0; esz = 16; break;
    case RTS_DBG_PCI_SE: src = c->d.SE; count = pci ? n : 0; esz = 1; break;
    case RTS_DBG_PCI_OB: src = c->d.OB; count = pci ? nb : 0; esz = 1; break;
    case RTS_DBG_PCI_DILATED: src = c->d.DILATED; count = pci ? nb : 0; esz = 1; break;
    case RTS_DBG_PCI_LISTS: {
      const size_t w = pci ? (size_t)c->prm.nbr_cap : 0;
      count = pci ? n * (w + 1) : 0;
      if (n_out) *n_out = count;
      if (count * 4 > cap) return fail(c, RTS_E_CAPACITY, "debug view needs %zu bytes", count * 4);
      if (count) {
        launch_pci_lists_rows(c->prm, c->d, (uint32_t *)d_out, c->stream);
        HIP_OK(c, hipGetLastError());
        HIP_OK(c, hipMemcpyAsync((uint32_t *)d_out + n * w, c->d.NNB, n * 4,
                                 hipMemcpyDeviceToDevice, c->stream));
      }
      return RTS_OK;
    }
    case RTS_DBG_OCCUPIED: {
      DevScalars S;
      HIP_OK(c, hipMemcpyAsync(&S, c->d.S, sizeof(S), hipMemcpyDeviceToHost, c->stream));
      HIP_OK(c, hipStreamSynchronize(c->stream));
      src = c->d.OCC;
      count = S.n_occ;
      break;
    }
    default: return fail(c, RTS_E_INVALID, "unknown debug view %d", what);
  }
  if (n_out) *n_out = count;
  if (count * esz > cap) return fail(c, RTS_E_CAPACITY, "debug view needs %zu bytes", count * esz);
  if (count) HIP_OK(c, hipMemcpyAsync(d_out, src, count * esz, hipMemcpyDeviceToDevice, c->stream));
  return RTS_OK;
}

rts_status rts_get_tune(rts_ctx *c, rts_tune *out) {
  if (!c || !out) return RTS_E_INVALID;
  out->grid_wave = c->grid_wave;
  out->grid_search = c->grid_search;
  out->grid_force = c->grid_force;
  out->search_threads = c->search_threads;
  out->force_lanes = c->force_lanes;
  out->force_threads = 512;
  out->candidates = c->tune_candidates;
  out->ms_per_step = c->tune_ms;
  return RTS_OK;
}

rts_status rts_set_tune(rts_ctx *c, const rts_tune *t) {
  if (!c || !t) return RTS_E_INVALID;
  if (t->grid_wave < 1 || t->grid_search < 1 || t->grid_force < 1 ||
      (t->search_threads != 256 && t->search_threads != 512) ||
      (t->force_lanes != 4 && t->force_lanes != 8) ||
      (t->force_threads != 0 && t->force_threads != 512))
    return fail(c, RTS_E_INVALID, "launch shape out of range");
  c->grid_wave = t->grid_wave;
  c->grid_search = t->grid_search;
  c->grid_force = t->grid_force;
  c->search_threads = t->search_threads;
  c->force_lanes = t->force_lanes;
  destroy_graphs(c);  // the next advance captures the new shape
  return RTS_OK;
}

rts_status rts_autotune(rts_ctx *c, int32_t steps, void *d_scratch, size_t scratch_bytes,
                        rts_tune *out) {
  if (c) c->fresh = false;
  if (!c || steps < 1 || !d_scratch) return RTS_E_INVALID;
  if (c->cfg.solver != RTS_WCSPH)
    return fail(c, RTS_E_UNSUPPORTED, "the launch shape is tuned for the WCSPH step");
  if (!c->has_state) return fail(c, RTS_E_STATE, "no state");
  if (c->poisoned) return fail(c, RTS_E_STATE, "state failed; set or load a state first");
  size_t need = 0;
  rts_state_bytes(c, &need);
  if (scratch_bytes < need)
    return fail(c, RTS_E_CAPACITY, "scratch holds %zu of %zu bytes", scratch_bytes, need);
  rts_status s = rts_save_state(c, d_scratch, scratch_bytes);
  if (s) return s;
  int dev = 0;
  HIP_OK(c, hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIP_OK(c, hipGetDeviceProperties(&prop, dev));
  const int cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  // The launch shape is tuned one kernel group at a time: the grid of the
  // one-wave-per-block kernels, then the search's workgroup size and count,
  // then the force's lanes per particle and workgroup count, each against
  // the best of the ones before.  No choice changes any result.
  const int wave_m[] = {4, 8};
  const int search_t[] = {512, 256};
  const int search_m[] = {2, 3, 4, 6};
  const int force_l[] = {8, 4};
  const int force_m[] = {1, 2, 3, 4};
  struct Shape {
    int gw, gs, gf, st, fl;
  };
  Shape best{c->grid_wave, c->grid_search, c->grid_force, c->search_threads, c->force_lanes};
  double best_ms = INFINITY;
  int cand = 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  auto time_shape = [&](const Shape &sh) {
    c->grid_wave = sh.gw;
    c->grid_search = sh.gs;
    c->grid_force = sh.gf;
    c->search_threads = sh.st;
    c->force_lanes = sh.fl;
    destroy_graphs(c);
    if (c->cfg.use_graph) s = build_graphs(c);
    if (!s) s = rts_advance(c, 1);                 // first replay of the new shape
    if (!s) s = rts_load_state(c, d_scratch, need);
    if (s) return;
    he = hipEventRecord(e0, c->stream);
    if (he == hipSuccess) s = rts_advance(c, steps);
    if (!s && he == hipSuccess) he = hipEventRecord(e1, c->stream);
    if (!s && he == hipSuccess) he = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (!s && he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    if (s || he != hipSuccess) return;
    ++cand;
    if (ms < best_ms) {
      best_ms = ms;
      best = sh;
    }
    s = rts_load_state(c, d_scratch, need);
  };
  const auto ok = [&] { return !s && he == hipSuccess; };
  for (int a = 0; a < 2 && ok(); ++a) {
    Shape sh = best;
    sh.gw = cus * wave_m[a];
    time_shape(sh);
  }
  for (int t = 0; t < 2 && ok(); ++t)
    for (int m = 0; m < 4 && ok(); ++m) {
      Shape sh = best;
      sh.st = search_t[t];
      sh.gs = cus * search_m[m];
      time_shape(sh);
    }
  for (int l = 0; l < 2 && ok(); ++l)
    for (int m = 0; m < 4 && ok(); ++m) {
      Shape sh = best;
      sh.fl = force_l[l];
      sh.gf = cus * force_m[m];
      time_shape(sh);
    }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  c->grid_wave = best.gw;
  c->grid_search = best.gs;
  c->grid_force = best.gf;
  c->search_threads = best.st;
  c->force_lanes = best.fl;
  destroy_graphs(c);
  rts_status r = rts_load_state(c, d_scratch, need);
  if (s) return s;
  if (he != hipSuccess) return fail(c, RTS_E_DEVICE, "timing failed: %s", hipGetErrorString(he));
  if (r) return r;
  c->tune_candidates = cand;
  c->tune_ms = best_ms / steps;
  HIP_OK(c, hipStreamSynchronize(c->stream));
  if (out) return rts_get_tune(c, out);
  return RTS_OK;
}

namespace {
// Tape of the differentiable run: checkpoints, the frames of one segment,
// the adjoint arrays.
struct DiffTape {
  float4 *CKX, *CKV;       // checkpoints, n each
  float4 *FX, *FV;         // segment frames: state at the start of each substep
  float *FR, *FP;          // density, pressure of each frame
  float4 *XP, *VR;         // packed (x, p / rho^2), (v, rho) of the substep being advanced;
                           // in the adjoint, the frame's (x, rho), (v, p)
  uint32_t *FL, *FN;       // lists and counts of each frame
  float4 *TX, *TV;         // state after the segment's last substep
  float4 *XB, *VB, *AB;    // adjoints of x, v, a
  float4 *XRB;             // (x, adjoint of rho) of the frame being differentiated
  double *BB, *AA;         // per-particle parameter adjoints
  double *RED;             // their sums
};

size_t diff_carve(const rts_diff_desc &D, int64_t n, char *base, DiffTape *t) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char * {
    char *q = base ? base + off : nullptr;
    off += align256(bytes > 0 ? bytes : 1);
    return q;
  };
  const size_t nn = (size_t)(n > 0 ? n : 1);
  const size_t nck = (size_t)((D.n_sub + D.ckpt_every - 1) / D.ckpt_every);
  const size_t nf = (size_t)D.ckpt_every;
  DiffTape u;
  u.CKX = (float4 *)take(nck * nn * 16);
  u.CKV = (float4 *)take(nck * nn * 16);
  u.FX = (float4 *)take(nf * nn * 16);
  u.FV = (float4 *)take(nf * nn * 16);
  u.FR = (float *)take(nf * nn * 4);
  u.FP = (float *)take(nf * nn * 4);
  u.FL = (uint32_t *)take(nf * nn * (size_t)D.list_cap * 4);
  u.FN = (uint32_t *)take(nf * nn * 4);
  u.XP = (float4 *)take(nn * 16);
  u.VR = (float4 *)take(nn * 16);
  u.TX = (float4 *)take(nn * 16);
  u.TV = (float4 *)take(nn * 16);
  u.XB = (float4 *)take(nn * 16);
  u.VB = (float4 *)take(nn * 16);
  u.AB = (float4 *)take(nn * 16);
  u.XRB = (float4 *)take(nn * 16);
  u.BB = (double *)take(nn * 8);
  u.AA = (double *)take(nn * 8);
  u.RED = (double *)take(16);
  if (t) *t = u;
  return off;
}

rts_status diff_check(rts_ctx *c, const rts_diff_desc *D, int64_t n) {
  if (!c || !D) return RTS_E_INVALID;
  if (c->cfg.solver != RTS_WCSPH)
    return fail(c, RTS_E_UNSUPPORTED, "the differentiable substep is WCSPH");
  if (D->n_sub < 1 || D->ckpt_every < 1 || D->list_cap < 8 || D->list_cap > 4096 ||
      !(D->dt > 0) || !(D->B > 0) || !(D->alpha > 0))
    return fail(c, RTS_E_INVALID, "bad differentiable-run description");
  if (n < 0 || n > c->ncap) return fail(c, RTS_E_CAPACITY, "n %lld exceeds capacity", (long long)n);
  return RTS_OK;
}

// Forward substeps k0..k1 from (X0, V0): frames (when kept) and the end state.
void diff_run_segment(rts_ctx *c, const rts_diff_desc &D, int n, const DiffTape &t,
                      const float4 *X0, const float4 *V0, int len, bool keep, float4 *Xend,
                      float4 *Vend) {
  const float hc0 = (float)(c->cfg.h * c->cfg.c0);
  const size_t nn = (size_t)(n > 0 ? n : 1);
  const float4 *X = X0, *V = V0;
  for (int k = 0; k < len; ++k) {
    const size_t f = keep ? (size_t)k : 0;
    float4 *fx = t.FX + f * nn, *fv = t.FV + f * nn;
    if (X != fx) {
      (void)hipMemcpyAsync(fx, X, nn * 16, hipMemcpyDeviceToDevice, c->stream);
      (void)hipMemcpyAsync(fv, V, nn * 16, hipMemcpyDeviceToDevice, c->stream);
    }
    uint32_t *L = t.FL + f * nn * (size_t)D.list_cap, *NN = t.FN + f * nn;
    float *R = t.FR + f * nn, *P = t.FP + f * nn;
    launch_diff_setup(c->prm, c->d, n, D.list_cap, (float)D.B, fx, fv, L, NN, R, P, t.XP, t.VR,
                      c->grid_wave, c->stream);
    // the next state never aliases the frame being read: without kept frames
    // it goes to TX / TV and is copied into frame 0 by the next substep
    const bool last = k + 1 == len;
    float4 *xn = last ? Xend : (keep ? t.FX + (f + 1) * nn : t.TX);
    float4 *vn = last ? Vend : (keep ? t.FV + (f + 1) * nn : t.TV);
    launch_diff_force_euler(c->prm, c->d, n, D.list_cap, (float)D.dt, (float)D.alpha, hc0, t.XP,
                            t.VR, L, NN, xn, vn, c->stream);
    X = xn;
    V = vn;
  }
}

}  // namespace

rts_status rts_diff_tape_bytes(rts_ctx *c, const rts_diff_desc *D, int64_t n, size_t *bytes) {
  rts_status s = diff_check(c, D, n);
  if (s) return s;
  if (!bytes) return RTS_E_INVALID;
  *bytes = diff_carve(*D, n, nullptr, nullptr);
  return RTS_OK;
}

rts_status rts_diff_forward(rts_ctx *c, const rts_diff_desc *D, int64_t n, const float *d_x0,
                            const float *d_v0, float *d_xT, float *d_vT, void *d_tape,
                            size_t tape_bytes) {
  rts_status s = diff_check(c, D, n);
  if (s) return s;
  if (n > 0 && (!d_x0 || !d_v0 || !d_xT || !d_vT)) return fail(c, RTS_E_INVALID, "NULL array");
  if (!d_tape || tape_bytes < diff_carve(*D, n, nullptr, nullptr) || ((uintptr_t)d_tape & 255u))
    return fail(c, RTS_E_CAPACITY, "tape too small or not 256-byte aligned");
  rts_status u = unbin(c);  // the substeps sort with the context's arrays
  if (u) return u;
  DiffTape t;
  diff_carve(*D, n, (char *)d_tape, &t);
  c->prm.n = (int32_t)n;
  c->cur = 0;
  c->has_state = false;   // the particle buffers serve as scratch
  c->fresh = false;
  destroy_graphs(c);
  launch_reset_scalars(c->d.S, c->stream);
  const size_t nn = (size_t)(n > 0 ? n : 1);
  launch_diff_planes_in((int)n, d_x0, t.CKX, c->stream);
  launch_diff_planes_in((int)n, d_v0, t.CKV, c->stream);
  const int nck = (D->n_sub + D->ckpt_every - 1) / D->ckpt_every;
  for (int q = 0; q < nck; ++q) {
    const int len = q + 1 < nck ? D->ckpt_every : D->n_sub - q * D->ckpt_every;
    // the final state goes to the (not yet used) adjoint buffers
    float4 *xe = q + 1 < nck ? t.CKX + (size_t)(q + 1) * nn : t.XB;
    float4 *ve = q + 1 < nck ? t.CKV + (size_t)(q + 1) * nn : t.VB;
    diff_run_segment(c, *D, (int)n, t, t.CKX + (size_t)q * nn, t.CKV + (size_t)q * nn, len, false,
                     xe, ve);
    if (q + 1 == nck) {
      launch_diff_planes_out((int)n, xe, d_xT, c->stream);
      launch_diff_planes_out((int)n, ve, d_vT, c->stream);
    }
  }
  HIP_OK(c, hipGetLastError());
  return RTS_OK;
}

rts_status rts_diff_backward(rts_ctx *c, const rts_diff_desc *D, int64_t n,
                             const float *d_xT_bar, const float *d_vT_bar, float *d_x0_bar,
                             float *d_v0_bar, double *h_B_bar, double *h_alpha_bar, void *d_tape,
                             size_t tape_bytes) {
  rts_status s = diff_check(c, D, n);
  if (s) return s;
  if (n > 0 && !d_xT_bar) return fail(c, RTS_E_INVALID, "NULL dL/dx(T)");
  if (!d_tape || tape_bytes < diff_carve(*D, n, nullptr, nullptr) || ((uintptr_t)d_tape & 255u))
    return fail(c, RTS_E_CAPACITY, "tape too small or not 256-byte aligned");
  rts_status u = unbin(c);  // the substeps sort with the context's arrays
  if (u) return u;
  DiffTape t;
  diff_carve(*D, n, (char *)d_tape, &t);
  c->prm.n = (int32_t)n;
  c->cur = 0;
  c->has_state = false;
  destroy_graphs(c);
  const size_t nn = (size_t)(n > 0 ? n : 1);
  const float hc0 = (float)(c->cfg.h * c->cfg.c0);
  launch_diff_planes_in((int)n, d_xT_bar, t.XB, c->stream);
  if (d_vT_bar) {
    launch_diff_planes_in((int)n, d_vT_bar, t.VB, c->stream);
    launch_diff_zero((int)n, nullptr, t.BB, t.AA, c->stream);
  } else {
    launch_diff_zero((int)n, t.VB, t.BB, t.AA, c->stream);
  }
  const int nck = (D->n_sub + D->ckpt_every - 1) / D->ckpt_every;
  for (int q = nck - 1; q >= 0; --q) {
    const int len = q + 1 < nck ? D->ckpt_every : D->n_sub - q * D->ckpt_every;
    // recompute the segment, keeping every frame (the end state is not needed)
    diff_run_segment(c, *D, (int)n, t, t.CKX + (size_t)q * nn, t.CKV + (size_t)q * nn, len, true,
                     t.TX, t.TV);
    for (int k = len - 1; k >= 0; --k) {
      const size_t f = (size_t)k;
      launch_diff_adjoint(c->prm, c->d, (int)n, D->list_cap, (float)D->dt, (float)D->B,
                          (float)D->alpha, hc0, t.FX + f * nn, t.FV + f * nn, t.FR + f * nn,
                          t.FP + f * nn, t.FL + f * nn * (size_t)D->list_cap, t.FN + f * nn,
                          t.XB, t.VB, t.AB, t.XP, t.VR, t.XRB, t.BB, t.AA, c->stream);
    }
  }
  if (d_x0_bar) launch_diff_planes_out((int)n, t.XB, d_x0_bar, c->stream);
  if (d_v0_bar) launch_diff_planes_out((int)n, t.VB, d_v0_bar, c->stream);
  launch_diff_reduce((int)n, t.BB, t.AA, t.RED, c->stream);
  HIP_OK(c, hipGetLastError());
  double red[2] = {0.0, 0.0};
  HIP_OK(c, hipMemcpyAsync(red, t.RED, 16, hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  if (h_B_bar) *h_B_bar = red[0];
  if (h_alpha_bar) *h_alpha_bar = red[1];
  DevScalars S;
  HIP_OK(c, hipMemcpy(&S, c->d.S, sizeof(S), hipMemcpyDeviceToHost));
  if (S.status) return fail(c, (rts_status)S.status, "device reported %s during the run",
                            rts_status_string((rts_status)S.status));
  return RTS_OK;
}

rts_status rts_grid_info(rts_ctx *c, int32_t *nc3, int64_t *nblocks, double *mass, double *B,
                         double *dt_base) {
  if (!c) return RTS_E_INVALID;
  if (nc3) for (int d = 0; d < 3; ++d) nc3[d] = c->prm.nc[d];
  if (nblocks) *nblocks = c->prm.nb;
  if (mass) *mass = c->mass;
  if (B) *B = c->B;
  if (dt_base) *dt_base = c->dt_base;
  return RTS_OK;
}

}  // extern "C"
