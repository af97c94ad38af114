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
    ]


class OrcInfo(C.Structure):
    _fields_ = [
        ("nc", C.c_int32 * 3), ("nblocks", C.c_int64), ("o", C.c_float * 3),
        ("inv_e", C.c_float), ("r2f", C.c_float), ("mass", C.c_double), ("B", C.c_double),
        ("sigma", C.c_double), ("dt_base", C.c_double),
        ("TV", C.c_float * MAX_LEVELS), ("TA", C.c_float * MAX_LEVELS), ("lmax", C.c_int32),
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
    L.orc_flags.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_neighbors.argtypes = [cfgp, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                C.c_int32, C.c_void_p, C.c_void_p]
    L.orc_density.argtypes = [cfgp, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                              C.c_void_p, C.c_void_p]
    L.orc_forces.argtypes = [cfgp, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                             C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
    L.orc_serna_predict.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double]
    L.orc_serna_correct.argtypes = [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p]
    L.orc_wcsph_step.argtypes = [cfgp, _p(OrcState)]
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


def flags(key, blk, level, validity):
    key = np.ascontiguousarray(key, np.uint32)
    blk = np.ascontiguousarray(blk, np.uint8)
    level = np.array(level, np.int32, copy=True)
    validity = np.array(validity, np.int32, copy=True)
    compute = np.zeros(key.shape[0], np.uint8)
    lib().orc_flags(key.shape[0], _ptr(key), _ptr(blk), _ptr(level), _ptr(validity), _ptr(compute))
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


def forces(cfg, x, v, rho, p, walls=None, which=None):
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 3)
    v = np.ascontiguousarray(v, np.float64).reshape(-1, 3)
    rho = np.ascontiguousarray(rho, np.float64)
    p = np.ascontiguousarray(p, np.float64)
    wx = np.zeros((0, 3)) if walls is None else np.ascontiguousarray(walls, np.float64).reshape(-1, 3)
    acc = np.zeros_like(x)
    w = None if which is None else np.ascontiguousarray(which, np.uint8)
    st = lib().orc_forces(C.byref(cfg), x.shape[0], _ptr(x), _ptr(v), _ptr(rho), _ptr(p),
                          wx.shape[0], _ptr(wx), None if w is None else _ptr(w), _ptr(acc))
    if st:
        raise RuntimeError(f"oracle forces status {st}")
    return acc


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
