"""ctypes binding of the CPU oracle (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never does.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "librts_oracle.so")
_lib = None

MAX_LEVELS = 8
WALL_BIT = 0x80000000
EMPTY_BLOCK = 0xFF
MODES = {"rts": 0, "global_fixed": 1, "global_adaptive": 2}


class OrcCfg(C.Structure):
    _fields_ = [
        ("spacing", C.c_double), ("h", C.c_double), ("support", C.c_double),
        ("block_edge", C.c_double), ("rho0", C.c_double), ("mass", C.c_double),
        ("c0", C.c_double), ("gamma", C.c_double), ("B", C.c_double),
        ("visc_alpha", C.c_double), ("visc_eps", C.c_double), ("g", C.c_double * 3),
        ("dom_min", C.c_double * 3), ("dom_max", C.c_double * 3), ("dt_base", C.c_double),
        ("r_crit", C.c_double),
        ("lambda_v", C.c_double), ("lambda_f", C.c_double), ("alpha_rts", C.c_double),
        ("beta2", C.c_double), ("beta_ratio", C.c_double),
        ("n_levels", C.c_int32), ("level_cap", C.c_int32), ("mode", C.c_int32),
        ("clamp_p", C.c_int32), ("serna_correct", C.c_int32), ("nbr_cap", C.c_int32),
        ("solver", C.c_int32), ("n_minor", C.c_int32), ("it_min", C.c_int32),
        ("it_max", C.c_int32), ("expand_layers", C.c_int32), ("local_fail", C.c_int32),
        ("global_limit", C.c_int32), ("short_majors", C.c_int32), ("two_ring_levels", C.c_int32),
        ("eta", C.c_double), ("eta_T", C.c_double), ("delta", C.c_double), ("r_list", C.c_double),
        ("adapt_dt", C.c_int32), ("grow_iters", C.c_int32), ("shrink_iters", C.c_int32),
        ("pad_adapt", C.c_int32), ("dt_min", C.c_double),
        ("dt_max", C.c_double), ("grow", C.c_double), ("shrink", C.c_double),
        ("phase_align", C.c_int32), ("pad_phase", C.c_int32),
    ]


class OrcInfo(C.Structure):
    _fields_ = [
        ("nc", C.c_int32 * 3), ("nblocks", C.c_int64), ("o", C.c_float * 3),
        ("inv_e", C.c_float), ("r2f", C.c_float), ("mass", C.c_double), ("B", C.c_double),
        ("sigma", C.c_double), ("dt_base", C.c_double),
        ("TV", C.c_float * MAX_LEVELS), ("TA", C.c_float * MAX_LEVELS), ("lmax", C.c_int32),
        ("r2l", C.c_float), ("delta", C.c_double),
    ]


class OrcState(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("nw", C.c_int32),
        ("x", C.POINTER(C.c_double)), ("v", C.POINTER(C.c_double)), ("a", C.POINTER(C.c_double)),
        ("rho", C.POINTER(C.c_double)), ("p", C.POINTER(C.c_double)),
        ("level", C.POINTER(C.c_int32)), ("validity", C.POINTER(C.c_int32)),
        ("age", C.POINTER(C.c_int32)), ("compute", C.POINTER(C.c_uint8)),
        ("wx", C.POINTER(C.c_double)),
        ("t", C.c_double), ("dt_prev", C.c_double), ("step", C.c_int64),
        ("n_active", C.c_int32), ("n_inter", C.c_int64), ("err_max", C.c_double),
        ("hist", C.c_int32 * MAX_LEVELS),
    ]


class OrcPciState(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("nw", C.c_int32),
        ("x", C.c_void_p), ("v", C.c_void_p), ("fvg", C.c_void_p), ("fp", C.c_void_p),
        ("p", C.c_void_p), ("rho", C.c_void_p), ("err", C.c_void_p),
        ("region", C.c_void_p), ("validity", C.c_void_p),
        ("compute", C.c_void_p), ("in_se", C.c_void_p), ("id", C.c_void_p), ("key", C.c_void_p),
        ("nbr", C.c_void_p), ("nnb", C.c_void_p),
        ("cell_start", C.c_void_p), ("blk_level", C.c_void_p), ("blk_ob", C.c_void_p),
        ("wx", C.c_void_p), ("wcell_start", C.c_void_p),
        ("major_len", C.c_int32), ("minor_in_major", C.c_int32), ("clean_majors", C.c_int32),
        ("major_excess", C.c_int32),
        ("minor_steps", C.c_int64), ("t", C.c_double),
        ("last_iters", C.c_int32), ("last_global_iters", C.c_int32), ("last_resets", C.c_int32),
        ("last_reverts", C.c_int32), ("last_early_end", C.c_int32), ("last_lists", C.c_int32),
        ("evals_density", C.c_int64), ("evals_force", C.c_int64),
        ("last_errmax", C.c_double), ("last_avg", C.c_double), ("hist", C.c_int32 * 4),
        ("dt_cur", C.c_double), ("last_dt", C.c_double), ("peak_iters", C.c_int32),
        ("pad_", C.c_int32), ("last_v2max", C.c_float), ("last_a2max", C.c_float),
        ("snap", C.c_void_p), ("snap_id", C.c_void_p), ("snap_t", C.c_double),
        ("snap_steps", C.c_int64), ("snap_major_len", C.c_int32), ("snap_clean", C.c_int32),
        ("rollbacks", C.c_int32), ("last_rollback", C.c_int32),
        ("trace", C.c_void_p), ("trace_p", C.c_void_p), ("trace_e", C.c_void_p),
        ("trace_cap", C.c_int32),
        ("trace_len", C.c_int32),
    ]


class OrcPciCtl(C.Structure):
    _fields_ = [
        ("iter", C.c_int32), ("row", C.c_int32), ("min_iter", C.c_int32), ("global_", C.c_int32),
        ("local_iters", C.c_int32), ("global_iters", C.c_int32), ("resets", C.c_int32),
        ("reverts", C.c_int32), ("local_off", C.c_int32),
    ]


class OrcPciIterRec(C.Structure):
    _fields_ = [
        ("iter", C.c_int32), ("row", C.c_int32), ("global_", C.c_int32), ("turn", C.c_uint32),
        ("action", C.c_int32), ("n_density", C.c_int32), ("n_force", C.c_int32),
        ("n_se", C.c_int32), ("errmax", C.c_double), ("avg", C.c_double),
    ]


CTL_KEEP, CTL_BACKUP, CTL_RESTORE = 0, 1, 2


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = C.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


def _p(t):
    return C.POINTER(t)


def _declare(L):
    cfgp = _p(OrcCfg)
    L.orc_derive.argtypes = [cfgp, _p(OrcInfo)]
    L.orc_kernel_W.argtypes = [cfgp, C.c_double]
    L.orc_kernel_W.restype = C.c_double
    L.orc_kernel_dWdr.argtypes = [cfgp, C.c_double]
    L.orc_kernel_dWdr.restype = C.c_double
    L.orc_lattice_sum.argtypes = [cfgp]
    L.orc_lattice_sum.restype = C.c_double
    L.orc_eos.argtypes = [cfgp, C.c_double]
    L.orc_eos.restype = C.c_double
    L.orc_keys.argtypes = [cfgp, C.c_int32, C.c_void_p, C.c_void_p]
    L.orc_sort.argtypes = [C.c_int64, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_block_levels.argtypes = [cfgp, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_rmin.argtypes = [cfgp, C.c_void_p, C.c_void_p]
    L.orc_flags.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                            C.c_int64, C.c_int32]
    L.orc_neighbors.argtypes = [cfgp, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                C.c_int32, C.c_void_p, C.c_void_p]
    L.orc_density.argtypes = [cfgp, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                              C.c_void_p, C.c_void_p]
    L.orc_forces.argtypes = [cfgp, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                             C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_forces_terms.argtypes = [cfgp, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p]
    L.orc_serna_predict.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double]
    L.orc_serna_correct.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p]
    L.orc_wcsph_step.argtypes = [cfgp, _p(OrcState)]
    vp = C.c_void_p
    L.orc_pci_delta.argtypes = [cfgp]
    L.orc_pci_delta.restype = C.c_double
    L.orc_pci_regions.argtypes = [cfgp, C.c_int32, vp, vp, vp, vp, vp, vp]
    L.orc_pci_dilate.argtypes = [cfgp, vp, vp, C.c_int, C.c_int]
    L.orc_pci_observed.argtypes = [cfgp, vp, vp]
    L.orc_pci_lists.argtypes = [cfgp, C.c_int32, vp, vp, vp, C.c_int32, vp, vp, vp, vp, C.c_int32,
                                vp, vp]
    L.orc_pci_density.argtypes = [cfgp, C.c_int32, vp, vp, vp, vp, vp, vp]
    L.orc_pci_pressure_force.argtypes = [cfgp, C.c_int32, vp, vp, vp, vp, vp, vp, vp, vp]
    L.orc_pci_pressure_force_terms.argtypes = [cfgp, C.c_int32, vp, vp, vp, vp, vp, vp, vp, vp,
                                               vp]
    L.orc_pci_nonpressure.argtypes = [cfgp, C.c_int32, vp, vp, vp, vp, vp, vp, vp]
    L.orc_pci_turn.argtypes = [C.c_int32, C.c_int32]
    L.orc_pci_turn.restype = C.c_uint32
    L.orc_pci_step.argtypes = [cfgp, _p(OrcPciState)]
    L.orc_pci_next_dt.argtypes = [cfgp, C.c_double, C.c_int32, C.c_int32, C.c_float, C.c_float]
    L.orc_pci_next_dt.restype = C.c_double
    L.orc_pci_major_begin.argtypes = [cfgp, _p(OrcPciState)]
    ctlp = _p(OrcPciCtl)
    L.orc_pci_ctl_init.argtypes = [cfgp, ctlp]
    L.orc_pci_ctl_more.argtypes = [cfgp, ctlp, C.c_double]
    L.orc_pci_ctl_more.restype = C.c_int
    L.orc_pci_ctl_turn.argtypes = [ctlp, C.c_int32, C.c_int32]
    L.orc_pci_ctl_turn.restype = C.c_uint32
    L.orc_pci_ctl_after.argtypes = [cfgp, ctlp, C.c_int32, C.c_double, C.c_double]
    L.orc_pci_ctl_after.restype = C.c_int
    L.orc_pci_major_length.argtypes = [cfgp, _p(OrcPciState), C.c_int32, C.c_int32]
    L.orc_pci_major_length.restype = C.c_int
    L.orc_pci_smaller_steps.argtypes = [cfgp, C.c_int32, vp, vp, vp, C.c_int32, vp, vp, vp, vp,
                                        vp]
    L.orc_pci_smaller_steps.restype = C.c_int
    L.orc_pci_region_validity.argtypes = [C.c_int32, C.c_int32]
    L.orc_pci_region_validity.restype = C.c_int32
    L.orc_adaptive_dt.argtypes = [cfgp, C.c_int32, vp]
    L.orc_adaptive_dt.restype = C.c_double
    L.orc_diff_run.argtypes = [cfgp, C.c_int32, vp, vp, C.c_int32, vp, C.c_double, C.c_double,
                               C.c_double, C.c_int32, vp, vp]
    L.orc_diff_grad.argtypes = [cfgp, C.c_int32, vp, vp, C.c_int32, vp, C.c_double, C.c_double,
                                C.c_double, C.c_int32, vp, vp, vp, vp, vp, vp]
    L.orc_num_threads.restype = C.c_int


def cfg_from_params(p: dict, **over) -> OrcCfg:
    q = dict(p)
    q.update(over)
    c = OrcCfg()
    c.spacing, c.h, c.support, c.block_edge = q["spacing"], q["h"], q["support"], q["block_edge"]
    c.rho0, c.mass = q["rho0"], q.get("mass", 0.0)
    c.c0, c.gamma, c.B = q["c0"], q["gamma"], q.get("B", 0.0)
    c.visc_alpha, c.visc_eps = q["visc_alpha"], q["visc_eps"]
    for d in range(3):
        c.g[d] = q["gravity"][d]
        c.dom_min[d] = q["domain_min"][d]
        c.dom_max[d] = q["domain_max"][d]
    c.dt_base = q["dt_base"]
    c.r_crit = q.get("r_crit", 0.0)
    c.lambda_v, c.lambda_f, c.alpha_rts = q["lambda_v"], q["lambda_f"], q["alpha_rts"]
    c.beta2, c.beta_ratio = q["beta2"], q["beta_ratio"]
    c.n_levels, c.level_cap = q["n_levels"], q["level_cap"]
    c.mode = MODES[q["mode"]] if isinstance(q["mode"], str) else int(q["mode"])
    c.clamp_p, c.serna_correct = q["clamp_p"], q["serna_correct"]
    c.nbr_cap = q.get("nbr_cap", 512)
    c.solver = 1 if q.get("solver", "wcsph") == "pcisph" else 0
    c.n_minor, c.it_min, c.it_max = q.get("n_minor", 4), q.get("it_min", 3), q.get("it_max", 50)
    c.expand_layers = q.get("expand_layers", 4)
    c.local_fail, c.global_limit = q.get("local_fail", 3), q.get("global_limit", 6)
    c.short_majors = q.get("short_majors", 10)
    c.two_ring_levels = q.get("two_ring_levels", 1)
    c.eta, c.eta_T = q.get("eta", 0.01), q.get("eta_T", 0.0025)
    c.delta, c.r_list = q.get("delta", 0.0), q.get("r_list", 0.0)
    c.adapt_dt, c.grow_iters = int(q.get("pci_adapt_dt", 0)), int(q.get("pci_grow_iters", 0))
    c.shrink_iters = int(q.get("pci_shrink_iters", 0))
    c.dt_min, c.dt_max = q.get("pci_dt_min", 0.0), q.get("pci_dt_max", 0.0)
    c.grow, c.shrink = q.get("pci_grow", 1.02), q.get("pci_shrink", 0.95)
    c.phase_align = int(q.get("phase_align", 0))
    return c


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def derive(cfg: OrcCfg) -> OrcInfo:
    info = OrcInfo()
    st = lib().orc_derive(C.byref(cfg), C.byref(info))
    if st:
        raise ValueError(f"oracle rejected the configuration (status {st})")
    return info


def kernel_W(cfg, r):
    return lib().orc_kernel_W(C.byref(cfg), float(r))


def kernel_dWdr(cfg, r):
    return lib().orc_kernel_dWdr(C.byref(cfg), float(r))


def lattice_sum(cfg):
    return lib().orc_lattice_sum(C.byref(cfg))


def eos(cfg, rho):
    return lib().orc_eos(C.byref(cfg), float(rho))


def keys(cfg, pos_f32):
    pos = np.ascontiguousarray(pos_f32, np.float32).reshape(-1, 3)
    out = np.zeros(pos.shape[0], np.uint32)
    lib().orc_keys(C.byref(cfg), pos.shape[0], _ptr(pos), _ptr(out))
    return out


def sort(nblocks, key):
    key = np.ascontiguousarray(key, np.uint32)
    perm = np.zeros(key.shape[0], np.uint32)
    start = np.zeros(int(nblocks) + 1, np.uint32)
    st = lib().orc_sort(int(nblocks), key.shape[0], _ptr(key), _ptr(perm), _ptr(start))
    if st:
        raise ValueError("key out of range")
    return perm, start


def block_levels(cfg, key, vel_f32, acc_f32):
    info = derive(cfg)
    key = np.ascontiguousarray(key, np.uint32)
    v = np.ascontiguousarray(vel_f32, np.float32).reshape(-1, 3)
    a = np.ascontiguousarray(acc_f32, np.float32).reshape(-1, 3)
    out = np.zeros(info.nblocks, np.uint8)
    lib().orc_block_levels(C.byref(cfg), key.shape[0], _ptr(key), _ptr(v), _ptr(a), _ptr(out))
    return out


def rmin(cfg, lvl):
    lvl = np.ascontiguousarray(lvl, np.uint8)
    out = np.zeros_like(lvl)
    lib().orc_rmin(C.byref(cfg), _ptr(lvl), _ptr(out))
    return out


def flags(key, blk, level, validity, step=0, phase_align=0):
    """W5 at base step ``step``: (level, validity, compute)."""
    key = np.ascontiguousarray(key, np.uint32)
    blk = np.ascontiguousarray(blk, np.uint8)
    level = np.array(level, np.int32, copy=True)
    validity = np.array(validity, np.int32, copy=True)
    compute = np.zeros(key.shape[0], np.uint8)
    lib().orc_flags(key.shape[0], _ptr(key), _ptr(blk), _ptr(level), _ptr(validity),
                    _ptr(compute), int(step), int(phase_align))
    return level, validity, compute


def neighbors(cfg, pos_f32, wpos_f32=None, want=None, cap=512):
    pos = np.ascontiguousarray(pos_f32, np.float32).reshape(-1, 3)
    n = pos.shape[0]
    wpos = np.zeros((0, 3), np.float32) if wpos_f32 is None else \
        np.ascontiguousarray(wpos_f32, np.float32).reshape(-1, 3)
    w = None if want is None else np.ascontiguousarray(want, np.uint8)
    nbr = np.zeros((max(n, 1), cap), np.uint32)
    nnb = np.zeros(max(n, 1), np.int32)
    st = lib().orc_neighbors(C.byref(cfg), n, _ptr(pos), wpos.shape[0], _ptr(wpos),
                             None if w is None else _ptr(w), cap, _ptr(nbr), _ptr(nnb))
    return st, nbr[:n], nnb[:n]


def density(cfg, x, walls=None, which=None):
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 3)
    wx = np.zeros((0, 3)) if walls is None else np.ascontiguousarray(walls, np.float64).reshape(-1, 3)
    rho = np.zeros(x.shape[0])
    p = np.zeros(x.shape[0])
    w = None if which is None else np.ascontiguousarray(which, np.uint8)
    st = lib().orc_density(C.byref(cfg), x.shape[0], _ptr(x), wx.shape[0], _ptr(wx),
                           None if w is None else _ptr(w), _ptr(rho), _ptr(p))
    if st:
        raise RuntimeError(f"oracle density status {st}")
    return rho, p


def forces(cfg, x, v, rho, p, walls=None, which=None, term_sums=False):
    """Accelerations; with ``term_sums`` also |g| + sum_j |pair term| per particle."""
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 3)
    v = np.ascontiguousarray(v, np.float64).reshape(-1, 3)
    rho = np.ascontiguousarray(rho, np.float64)
    p = np.ascontiguousarray(p, np.float64)
    wx = np.zeros((0, 3)) if walls is None else np.ascontiguousarray(walls, np.float64).reshape(-1, 3)
    acc = np.zeros_like(x)
    tsum = np.zeros(x.shape[0])
    w = None if which is None else np.ascontiguousarray(which, np.uint8)
    st = lib().orc_forces_terms(C.byref(cfg), x.shape[0], _ptr(x), _ptr(v), _ptr(rho), _ptr(p),
                                wx.shape[0], _ptr(wx), None if w is None else _ptr(w), _ptr(acc),
                                _ptr(tsum))
    if st:
        raise RuntimeError(f"oracle forces status {st}")
    return (acc, tsum) if term_sums else acc


def serna_predict(x, v, a, dt):
    lib().orc_serna_predict(x.shape[0], _ptr(x), _ptr(v), _ptr(a), float(dt))


def serna_correct(x, v, a, a_new, dtau, which=None):
    w = None if which is None else np.ascontiguousarray(which, np.uint8)
    lib().orc_serna_correct(x.shape[0], _ptr(x), _ptr(v), _ptr(a), _ptr(a_new),
                            _ptr(np.ascontiguousarray(dtau, np.float64)),
                            None if w is None else _ptr(w))


class WCSPH:
    """FP64 oracle run of Algorithm 1 (or a global comparator) on one scene."""

    def __init__(self, params: dict, pos, vel=None, walls=None, **over):
        self.cfg = cfg_from_params(params, **over)
        self.info = derive(self.cfg)
        n = int(np.asarray(pos).reshape(-1, 3).shape[0])
        self.x = np.array(np.asarray(pos, np.float64).reshape(-1, 3), copy=True)
        self.v = np.zeros((n, 3)) if vel is None else np.array(np.asarray(vel, np.float64).reshape(-1, 3))
        self.a = np.zeros((n, 3))
        self.rho = np.full(n, self.cfg.rho0)
        self.p = np.zeros(n)
        self.level = np.full(n, 0xF, np.int32)
        self.validity = np.zeros(n, np.int32)
        self.age = np.zeros(n, np.int32)
        self.compute = np.zeros(n, np.uint8)
        self.walls = np.zeros((0, 3)) if walls is None else \
            np.ascontiguousarray(np.asarray(walls, np.float64).reshape(-1, 3))
        self.state = OrcState()
        s = self.state
        s.n, s.nw = n, self.walls.shape[0]
        dp = C.POINTER(C.c_double)
        s.x = self.x.ctypes.data_as(dp)
        s.v = self.v.ctypes.data_as(dp)
        s.a = self.a.ctypes.data_as(dp)
        s.rho = self.rho.ctypes.data_as(dp)
        s.p = self.p.ctypes.data_as(dp)
        ip = C.POINTER(C.c_int32)
        s.level = self.level.ctypes.data_as(ip)
        s.validity = self.validity.ctypes.data_as(ip)
        s.age = self.age.ctypes.data_as(ip)
        s.compute = self.compute.ctypes.data_as(C.POINTER(C.c_uint8))
        s.wx = self.walls.ctypes.data_as(dp)
        s.t, s.dt_prev, s.step = 0.0, 0.0, 0
        self.history = []

    def step(self, n=1):
        for _ in range(n):
            st = lib().orc_wcsph_step(C.byref(self.cfg), C.byref(self.state))
            if st:
                raise RuntimeError(f"oracle step status {st} at step {self.state.step}")
            s = self.state
            self.history.append(dict(step=int(s.step), t=s.t, n_active=s.n_active,
                                     n_inter=int(s.n_inter), err_max=s.err_max,
                                     hist=list(s.hist)))
        return self

    @property
    def t(self):
        return self.state.t


def num_threads():
    return int(lib().orc_num_threads())


# ---------------------------------------------------------------------------
# PCISPH with regional iteration counts
# ---------------------------------------------------------------------------
def pci_delta(cfg):
    return lib().orc_pci_delta(C.byref(cfg))


def pci_next_dt(cfg, dt, peak_iters, excess, v2max, a2max):
    return lib().orc_pci_next_dt(C.byref(cfg), float(dt), int(peak_iters), int(excess),
                                 float(v2max), float(a2max))


def pci_turn(col, row):
    return int(lib().orc_pci_turn(int(col), int(row)))


class PciControl:
    """Algorithm 3's loop control on its own: feed it the errors after each
    iteration and read the decisions."""

    def __init__(self, cfg, standard=False):
        self.cfg = cfg
        self.standard = int(bool(standard))
        self.k = OrcPciCtl()
        lib().orc_pci_ctl_init(C.byref(cfg), C.byref(self.k))

    def more(self, errmax):
        return bool(lib().orc_pci_ctl_more(C.byref(self.cfg), C.byref(self.k), float(errmax)))

    def turn(self, col):
        return int(lib().orc_pci_ctl_turn(C.byref(self.k), int(col), self.standard))

    def after(self, errmax, avg):
        return int(lib().orc_pci_ctl_after(C.byref(self.cfg), C.byref(self.k), self.standard,
                                           float(errmax), float(avg)))

    def __getattr__(self, name):
        k = self.__dict__["k"]
        return getattr(k, "global_" if name == "global_" or name == "glob" else name)


def pci_major_length(cfg, state, global_iters, standard=False):
    """Ends a minor step in the major-step length controller; returns 1 when
    the major step ends.  ``state`` is an OrcPciState (only its major-step
    counters are used)."""
    return int(lib().orc_pci_major_length(C.byref(cfg), C.byref(state), int(global_iters),
                                          int(bool(standard))))


def pci_region_validity(region, major_len):
    return int(lib().orc_pci_region_validity(int(region), int(major_len)))


def pci_smaller_steps(cfg, key, vel_f32, acc_f32, major_len, region, validity, compute,
                      blk_level, blk_ob):
    """S7 on the given arrays (modified in place); returns 1 if a block changed."""
    key = np.ascontiguousarray(key, np.uint32)
    v = np.ascontiguousarray(vel_f32, np.float32).reshape(-1, 3)
    a = np.ascontiguousarray(acc_f32, np.float32).reshape(-1, 3)
    for arr, dt in ((region, np.int32), (validity, np.int32), (compute, np.uint8),
                    (blk_level, np.uint8), (blk_ob, np.uint8)):
        assert arr.dtype == dt and arr.flags.c_contiguous
    return int(lib().orc_pci_smaller_steps(C.byref(cfg), key.shape[0], _ptr(key), _ptr(v), _ptr(a),
                                           int(major_len), _ptr(region), _ptr(validity),
                                           _ptr(compute), _ptr(blk_level), _ptr(blk_ob)))


def adaptive_dt(cfg, acc):
    a = np.ascontiguousarray(acc, np.float64).reshape(-1, 3)
    return float(lib().orc_adaptive_dt(C.byref(cfg), a.shape[0], _ptr(a)))


def pci_regions(cfg, key, vel_f32, acc_f32):
    """(raw, lvl, observed) block arrays of a major step's region determination."""
    info = derive(cfg)
    key = np.ascontiguousarray(key, np.uint32)
    v = np.ascontiguousarray(vel_f32, np.float32).reshape(-1, 3)
    a = np.ascontiguousarray(acc_f32, np.float32).reshape(-1, 3)
    raw = np.zeros(info.nblocks, np.uint8)
    lvl = np.zeros(info.nblocks, np.uint8)
    ob = np.zeros(info.nblocks, np.uint8)
    lib().orc_pci_regions(C.byref(cfg), key.shape[0], _ptr(key), _ptr(v), _ptr(a), _ptr(raw),
                          _ptr(lvl), _ptr(ob))
    return raw, lvl, ob


def pci_dilate(cfg, lvl, level, layers):
    lvl = np.ascontiguousarray(lvl, np.uint8)
    out = np.zeros_like(lvl)
    lib().orc_pci_dilate(C.byref(cfg), _ptr(lvl), _ptr(out), int(level), int(layers))
    return out


def pci_observed(cfg, lvl):
    lvl = np.ascontiguousarray(lvl, np.uint8)
    out = np.zeros_like(lvl)
    lib().orc_pci_observed(C.byref(cfg), _ptr(lvl), _ptr(out))
    return out


def pci_lists(cfg, pos_f32, cell_start, key, wpos_f32, wcell_start, want=None, rings=None,
              cap=None):
    """Lists of sorted particles against a stored grid: (nbr (n, cap), nnb)."""
    pos = np.ascontiguousarray(pos_f32, np.float32).reshape(-1, 3)
    n = pos.shape[0]
    wpos = np.ascontiguousarray(wpos_f32, np.float32).reshape(-1, 3)
    cap = int(cap or cfg.nbr_cap)
    nbr = np.zeros((n, cap), np.uint32)
    nnb = np.zeros(n, np.int32)
    cs = np.ascontiguousarray(cell_start, np.uint32)
    ws = np.ascontiguousarray(wcell_start, np.uint32)
    key = np.ascontiguousarray(key, np.uint32)
    w = None if want is None else np.ascontiguousarray(want, np.uint8)
    r = None if rings is None else np.ascontiguousarray(rings, np.uint8)
    st = lib().orc_pci_lists(C.byref(cfg), n, _ptr(pos), _ptr(cs), _ptr(key), wpos.shape[0],
                             _ptr(wpos), _ptr(ws), _ptr(w) if w is not None else None,
                             _ptr(r) if r is not None else None, cap, _ptr(nbr), _ptr(nnb))
    return st, nbr, nnb


def _lists_arg(cfg, nbr, nnb):
    nbr = np.ascontiguousarray(nbr, np.uint32)
    assert nbr.shape[1] == cfg.nbr_cap
    return nbr, np.ascontiguousarray(nnb, np.int32)


def pci_density(cfg, xs, wx, nbr, nnb, which=None):
    xs = np.ascontiguousarray(xs, np.float64).reshape(-1, 3)
    wx = np.ascontiguousarray(wx, np.float64).reshape(-1, 3)
    nbr, nnb = _lists_arg(cfg, nbr, nnb)
    rho = np.zeros(xs.shape[0])
    w = None if which is None else np.ascontiguousarray(which, np.uint8)
    lib().orc_pci_density(C.byref(cfg), xs.shape[0], _ptr(xs), _ptr(wx), _ptr(nbr), _ptr(nnb),
                          _ptr(w) if w is not None else None, _ptr(rho))
    return rho


def pci_pressure_force(cfg, xs, wx, p, rho, nbr, nnb, which=None, term_sums=False):
    """Pressure accelerations; with ``term_sums`` also sum_j |pair term| per particle."""
    xs = np.ascontiguousarray(xs, np.float64).reshape(-1, 3)
    wx = np.ascontiguousarray(wx, np.float64).reshape(-1, 3)
    p = np.ascontiguousarray(p, np.float64)
    rho = np.ascontiguousarray(rho, np.float64)
    nbr, nnb = _lists_arg(cfg, nbr, nnb)
    fp = np.zeros_like(xs)
    tsum = np.zeros(xs.shape[0])
    w = None if which is None else np.ascontiguousarray(which, np.uint8)
    lib().orc_pci_pressure_force_terms(C.byref(cfg), xs.shape[0], _ptr(xs), _ptr(wx), _ptr(p),
                                       _ptr(rho), _ptr(nbr), _ptr(nnb),
                                       _ptr(w) if w is not None else None, _ptr(fp), _ptr(tsum))
    return (fp, tsum) if term_sums else fp


def pci_nonpressure(cfg, x, v, wx, nbr, nnb, which=None):
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 3)
    v = np.ascontiguousarray(v, np.float64).reshape(-1, 3)
    wx = np.ascontiguousarray(wx, np.float64).reshape(-1, 3)
    nbr, nnb = _lists_arg(cfg, nbr, nnb)
    out = np.zeros_like(x)
    w = None if which is None else np.ascontiguousarray(which, np.uint8)
    lib().orc_pci_nonpressure(C.byref(cfg), x.shape[0], _ptr(x), _ptr(v), _ptr(wx), _ptr(nbr),
                              _ptr(nnb), _ptr(w) if w is not None else None, _ptr(out))
    return out


def sorted_walls(cfg, walls):
    """Walls in their grid order (stable) and their block starts."""
    w32 = np.ascontiguousarray(walls, np.float32).reshape(-1, 3)
    info = derive(cfg)
    k = keys(cfg, w32)
    perm, start = sort(info.nblocks, k)
    return np.asarray(walls, np.float64).reshape(-1, 3)[perm], start, perm


class PCISPH:
    """FP64 oracle run of Algorithm 2 / 3 on one scene (arrays in block order)."""

    def __init__(self, params: dict, pos, vel=None, walls=None, **over):
        self.cfg = cfg_from_params(params, **over)
        self.info = derive(self.cfg)
        n = int(np.asarray(pos).reshape(-1, 3).shape[0])
        nb = int(self.info.nblocks)
        cap = int(self.cfg.nbr_cap)
        self.x = np.array(np.asarray(pos, np.float64).reshape(-1, 3), copy=True)
        self.v = np.zeros((n, 3)) if vel is None else np.array(np.asarray(vel, np.float64).reshape(-1, 3))
        self.fvg = np.zeros((n, 3))
        self.fp = np.zeros((n, 3))
        self.p = np.zeros(n)
        self.rho = np.full(n, self.cfg.rho0)
        self.err = np.zeros(n)
        self.region = np.ones(n, np.int32)
        self.validity = np.zeros(n, np.int32)
        self.compute = np.ones(n, np.uint8)
        self.in_se = np.zeros(n, np.uint8)
        self.id = np.arange(n, dtype=np.uint32)
        self.key = np.zeros(n, np.uint32)
        self.nbr = np.zeros((max(n, 1), cap), np.uint32)
        self.nnb = np.zeros(max(n, 1), np.int32)
        self.snap = np.zeros(15 * max(n, 1))
        self.snap_id = np.zeros(max(n, 1), np.uint32)
        self.cell_start = np.zeros(nb + 1, np.uint32)
        self.blk_level = np.full(nb, EMPTY_BLOCK, np.uint8)
        self.blk_ob = np.zeros(nb, np.uint8)
        walls = np.zeros((0, 3)) if walls is None else np.asarray(walls, np.float64).reshape(-1, 3)
        self.wx, self.wcell_start, self.wperm = sorted_walls(self.cfg, walls)
        self.wx = np.ascontiguousarray(self.wx)
        self.state = OrcPciState()
        s = self.state
        s.n, s.nw = n, self.wx.shape[0]
        for name in ("x", "v", "fvg", "fp", "p", "rho", "err", "region", "validity", "compute",
                     "in_se", "id", "key", "nbr", "nnb", "cell_start", "blk_level", "blk_ob",
                     "wx", "wcell_start", "snap", "snap_id"):
            setattr(s, name, _ptr(getattr(self, name)))
        s.major_len = int(self.cfg.n_minor)
        self.history = []
        self.trace = None
        self.trace_p = self.trace_e = None

    def enable_trace(self, cap=None, pressures=False, errors=False):
        """Record every correction iteration of each following minor step
        (``history[k]['trace']``), with the pressures after each iteration
        when ``pressures`` is set (``history[k]['trace_p']``, in block order)
        and the relative density errors of the particles each iteration
        evaluated (NaN for the others) when ``errors`` is set
        (``history[k]['trace_e']``)."""
        cap = int(cap if cap is not None else self.cfg.it_max)
        self.trace = (OrcPciIterRec * cap)()
        s = self.state
        s.trace = C.cast(self.trace, C.c_void_p)
        s.trace_cap = cap
        self.trace_p = np.zeros(cap * max(s.n, 1)) if pressures else None
        s.trace_p = _ptr(self.trace_p) if pressures else None
        self.trace_e = np.zeros(cap * max(s.n, 1)) if errors else None
        s.trace_e = _ptr(self.trace_e) if errors else None

    def step(self, n=1):
        """n accepted minor steps (a rolled-back major step does not count)."""
        s = self.state
        target = s.minor_steps + n
        while s.minor_steps < target:
            st = lib().orc_pci_step(C.byref(self.cfg), C.byref(self.state))
            if st:
                raise RuntimeError(f"oracle PCISPH step status {st}")
            self.history.append(dict(
                t=s.t, iters=s.last_iters, global_iters=s.last_global_iters,
                resets=s.last_resets, reverts=s.last_reverts, early_end=s.last_early_end,
                lists=s.last_lists, evals_density=s.evals_density, evals_force=s.evals_force,
                errmax=s.last_errmax, avg=s.last_avg, hist=list(s.hist),
                major_len=s.major_len, minor_in_major=s.minor_in_major, dt=s.last_dt,
                dt_next=s.dt_cur if s.dt_cur > 0 else self.cfg.dt_base,
                v2max=s.last_v2max, a2max=s.last_a2max, rollback=s.last_rollback,
                steps=s.minor_steps))
            if self.trace is not None:
                h = self.history[-1]
                h["trace"] = [dict(iter=r.iter, row=r.row, glob=r.global_, turn=r.turn,
                                   action=r.action, n_density=r.n_density, n_force=r.n_force,
                                   n_se=r.n_se, errmax=r.errmax, avg=r.avg)
                              for r in self.trace[:s.trace_len]]
                if self.trace_p is not None:
                    h["trace_p"] = self.trace_p[: s.trace_len * s.n].reshape(s.trace_len, s.n).copy()
                if self.trace_e is not None:
                    h["trace_e"] = self.trace_e[: s.trace_len * s.n].reshape(s.trace_len, s.n).copy()
        return self

    def major_begin(self):
        st = lib().orc_pci_major_begin(C.byref(self.cfg), C.byref(self.state))
        if st:
            raise RuntimeError(f"oracle major step set-up status {st}")

    @property
    def t(self):
        return self.state.t

    def in_caller_order(self, a):
        out = np.empty_like(a)
        out[self.id] = a
        return out


# ---------------------------------------------------------------------------
# differentiable WCSPH substeps
# ---------------------------------------------------------------------------
def diff_run(cfg, x0, v0, walls, B, alpha, dt, n_sub):
    x0 = np.ascontiguousarray(x0, np.float64).reshape(-1, 3)
    v0 = np.ascontiguousarray(v0, np.float64).reshape(-1, 3)
    w = np.ascontiguousarray(walls, np.float64).reshape(-1, 3)
    xo, vo = np.zeros_like(x0), np.zeros_like(v0)
    st = lib().orc_diff_run(C.byref(cfg), x0.shape[0], _ptr(x0), _ptr(v0), w.shape[0], _ptr(w),
                            float(B), float(alpha), float(dt), int(n_sub), _ptr(xo), _ptr(vo))
    if st:
        raise RuntimeError(f"oracle differentiable run status {st}")
    return xo, vo


def diff_grad(cfg, x0, v0, walls, B, alpha, dt, n_sub, xhat):
    """Loss mean_i |x_i(T) - xhat_i|^2 and its gradients (x0, v0, B, alpha)."""
    x0 = np.ascontiguousarray(x0, np.float64).reshape(-1, 3)
    v0 = np.ascontiguousarray(v0, np.float64).reshape(-1, 3)
    w = np.ascontiguousarray(walls, np.float64).reshape(-1, 3)
    xh = np.ascontiguousarray(xhat, np.float64).reshape(-1, 3)
    gx, gv = np.zeros_like(x0), np.zeros_like(v0)
    loss, gB, ga = C.c_double(0), C.c_double(0), C.c_double(0)
    st = lib().orc_diff_grad(C.byref(cfg), x0.shape[0], _ptr(x0), _ptr(v0), w.shape[0], _ptr(w),
                             float(B), float(alpha), float(dt), int(n_sub), _ptr(xh),
                             C.byref(loss), _ptr(gx), _ptr(gv), C.byref(gB), C.byref(ga))
    if st:
        raise RuntimeError(f"oracle differentiable gradient status {st}")
    return loss.value, gx, gv, gB.value, ga.value
