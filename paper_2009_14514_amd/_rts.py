"""ctypes binding of librts.so: argument marshalling only.

Every entry point of include/rts.h has a function of the same name here.
Device memory is plain integer addresses (torch tensors' data_ptr()).
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librts.so")

RTS_OK, RTS_E_INVALID, RTS_E_CAPACITY, RTS_E_DEVICE, RTS_E_NUMERICAL, RTS_E_STATE, \
    RTS_E_UNSUPPORTED = range(7)
STATUS_NAMES = {0: "ok", 1: "invalid", 2: "capacity", 3: "device", 4: "numerical", 5: "state",
                6: "unsupported"}
RTS_WCSPH, RTS_PCISPH = 0, 1
MODES = {"rts": 0, "global_fixed": 1, "global_adaptive": 2}
MAX_LEVELS = 8
DEBUG_NBR_ROW = 1024

DBG = {name: i for i, name in enumerate([
    "POS", "VEL", "ACC", "ACC_NEW", "META", "ID", "KEY", "PERM", "CELL_START", "BLK_LEVEL_RAW",
    "BLK_LEVEL", "NNB", "NBR", "PRESSURE", "PRE_POS", "PRE_VEL", "PRE_ACC", "PRE_META", "PRE_ID",
    "WALL_POS", "WALL_ID", "WALL_CELL_START", "OCCUPIED", "BLK_STATS",
    "PCI_XS", "PCI_PV", "PCI_FVG", "PCI_FP", "PCI_SE", "PCI_OB", "PCI_DILATED", "PCI_LISTS"])}

# exported symbols, in the order include/rts.h declares them
EXPORTS = [
    "rts_default_config", "rts_workspace_size", "rts_create", "rts_create_static",
    "rts_create_batch", "rts_destroy", "rts_set_walls", "rts_init_dam_break",
    "rts_get_scene_stats", "rts_get_scene_state",
    "rts_set_state", "rts_add_velocity", "rts_assign_levels", "rts_advance", "rts_sync",
    "rts_get_state", "rts_state_bytes", "rts_save_state", "rts_load_state", "rts_debug_get", "rts_grid_info",
    "rts_profile_advance", "rts_autotune", "rts_get_tune", "rts_set_tune", "rts_diff_tape_bytes",
    "rts_diff_forward", "rts_diff_backward", "rts_last_error", "rts_status_string",
]
PROF_KERNELS = ["key_hist", "scan", "scatter", "cell_gather", "rmin_flags", "search_density",
                "force", "step_stats", "correct_predict"]


class RtsConfig(C.Structure):
    _fields_ = [
        ("solver", C.c_int32), ("mode", C.c_int32), ("n_levels", C.c_int32),
        ("level_cap", C.c_int32), ("clamp_p", C.c_int32), ("serna_correct", C.c_int32),
        ("cand_cap", C.c_int32), ("use_graph", C.c_int32),
        ("spacing", C.c_double), ("h", C.c_double), ("support", C.c_double),
        ("block_edge", C.c_double), ("r_crit", C.c_double), ("rho0", C.c_double),
        ("mass", C.c_double), ("c0", C.c_double), ("gamma", C.c_double), ("B", C.c_double),
        ("visc_alpha", C.c_double), ("visc_eps", C.c_double), ("gravity", C.c_double * 3),
        ("domain_min", C.c_double * 3), ("domain_max", C.c_double * 3), ("dt_base", C.c_double),
        ("lambda_v", C.c_double), ("lambda_f", C.c_double), ("alpha_rts", C.c_double),
        ("beta2", C.c_double), ("beta_ratio", C.c_double),
        ("n_minor", C.c_int32), ("it_min", C.c_int32), ("it_max", C.c_int32),
        ("expand_layers", C.c_int32), ("local_fail", C.c_int32), ("global_limit", C.c_int32),
        ("short_majors", C.c_int32), ("nbr_cap", C.c_int32), ("two_ring_levels", C.c_int32),
        ("pci_adapt_dt", C.c_int32),
        ("eta", C.c_double), ("eta_T", C.c_double), ("delta", C.c_double), ("r_list", C.c_double),
        ("pci_grow_iters", C.c_int32), ("pci_shrink_iters", C.c_int32), ("pci_dt_min", C.c_double),
        ("pci_dt_max", C.c_double), ("pci_grow", C.c_double), ("pci_shrink", C.c_double),
        ("phase_align", C.c_int32), ("pad_", C.c_int32),
    ]


class RtsStats(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("time", C.c_double), ("dt_last", C.c_double),
        ("active_last", C.c_int64), ("inter_last", C.c_int64), ("active_total", C.c_int64),
        ("inter_total", C.c_int64), ("cand_total", C.c_int64), ("err_max_last", C.c_float),
        ("err_max_run", C.c_float),
        ("level_hist", C.c_int32 * MAX_LEVELS), ("nbr_max", C.c_int32), ("status", C.c_int32),
        ("bad_index", C.c_int32),
        ("pci_iters", C.c_int32), ("pci_global_iters", C.c_int32), ("pci_resets", C.c_int32),
        ("pci_reverts", C.c_int32), ("pci_early_end", C.c_int32), ("pci_lists", C.c_int32),
        ("pci_major_len", C.c_int32), ("pci_minor_in_major", C.c_int32),
        ("pci_errmax", C.c_double), ("pci_avg", C.c_double), ("pci_iters_total", C.c_int64),
        ("pci_rollbacks", C.c_int32), ("pci_pad", C.c_int32), ("pci_dt_next", C.c_double),
    ]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["level_hist"] = list(self.level_hist)
        return d


class RtsSceneStats(C.Structure):
    _fields_ = [("first", C.c_int64), ("n", C.c_int64), ("active_last", C.c_int64),
                ("inter_last", C.c_int64), ("err_max_last", C.c_float),
                ("level_hist", C.c_int32 * MAX_LEVELS), ("pad", C.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}
        d["level_hist"] = list(self.level_hist)
        return d


class RtsTune(C.Structure):
    _fields_ = [("grid_wave", C.c_int32), ("grid_search", C.c_int32), ("grid_force", C.c_int32),
                ("search_threads", C.c_int32), ("force_threads", C.c_int32),
                ("force_lanes", C.c_int32), ("candidates", C.c_int32), ("pad_", C.c_int32),
                ("ms_per_step", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad_"}


class RtsDiffDesc(C.Structure):
    _fields_ = [("n_sub", C.c_int32), ("ckpt_every", C.c_int32), ("list_cap", C.c_int32),
                ("pad", C.c_int32), ("dt", C.c_double), ("B", C.c_double), ("alpha", C.c_double)]


_lib = None


class RtsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def lib():
    """Loads librts.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        cfgp = C.POINTER(RtsConfig)
        L.rts_default_config.argtypes = [cfgp]
        L.rts_default_config.restype = None
        L.rts_workspace_size.argtypes = [cfgp, i64, i64, C.POINTER(C.c_size_t)]
        L.rts_create.argtypes = [cfgp, i64, i64, vp, C.c_size_t, vp, C.POINTER(vp)]
        L.rts_create_static.argtypes = [cfgp, i64, i64, vp, C.POINTER(vp)]
        L.rts_create_batch.argtypes = [cfgp, i32, vp, i64, vp, C.c_size_t, vp, C.POINTER(vp)]
        L.rts_init_dam_break.argtypes = [vp, i32, i64, vp, vp, C.c_double, C.c_double,
                                         C.c_uint64, C.c_uint64]
        L.rts_get_scene_stats.argtypes = [vp, C.POINTER(RtsSceneStats), i32]
        L.rts_get_scene_state.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
        L.rts_destroy.argtypes = [vp]
        L.rts_destroy.restype = None
        L.rts_set_walls.argtypes = [vp, vp, i64]
        L.rts_set_state.argtypes = [vp, vp, vp, i64]
        L.rts_add_velocity.argtypes = [vp, vp, i64]
        L.rts_assign_levels.argtypes = [vp, vp]
        L.rts_advance.argtypes = [vp, i32]
        L.rts_sync.argtypes = [vp, C.POINTER(RtsStats)]
        L.rts_get_state.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.rts_state_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
        L.rts_save_state.argtypes = [vp, vp, C.c_size_t]
        L.rts_load_state.argtypes = [vp, vp, C.c_size_t]
        L.rts_debug_get.argtypes = [vp, i32, vp, C.c_size_t, C.POINTER(C.c_size_t)]
        L.rts_grid_info.argtypes = [vp, vp, vp, vp, vp, vp]
        L.rts_profile_advance.argtypes = [vp, i32, C.POINTER(C.c_double)]
        L.rts_autotune.argtypes = [vp, i32, vp, C.c_size_t, C.POINTER(RtsTune)]
        L.rts_get_tune.argtypes = [vp, C.POINTER(RtsTune)]
        L.rts_set_tune.argtypes = [vp, C.POINTER(RtsTune)]
        dp = C.POINTER(RtsDiffDesc)
        L.rts_diff_tape_bytes.argtypes = [vp, dp, i64, C.POINTER(C.c_size_t)]
        L.rts_diff_forward.argtypes = [vp, dp, i64, vp, vp, vp, vp, vp, C.c_size_t]
        L.rts_diff_backward.argtypes = [vp, dp, i64, vp, vp, vp, vp, C.POINTER(C.c_double),
                                        C.POINTER(C.c_double), vp, C.c_size_t]
        L.rts_last_error.argtypes = [vp]
        L.rts_last_error.restype = C.c_char_p
        L.rts_status_string.argtypes = [C.c_int]
        L.rts_status_string.restype = C.c_char_p
        _lib = L
    return _lib


def check(status, ctx=None):
    if status != RTS_OK:
        msg = lib().rts_last_error(ctx).decode() if ctx else lib().rts_status_string(status).decode()
        raise RtsError(status, msg)


def default_config() -> RtsConfig:
    c = RtsConfig()
    lib().rts_default_config(C.byref(c))
    return c


def config_from_params(p: dict, **over) -> RtsConfig:
    """Maps a scene parameter dictionary onto rts_config."""
    q = dict(p)
    q.update(over)
    c = default_config()
    c.solver = RTS_PCISPH if q.get("solver", "wcsph") == "pcisph" else RTS_WCSPH
    mode = q.get("mode", "rts")
    c.mode = MODES[mode] if isinstance(mode, str) else int(mode)
    c.n_levels, c.level_cap = int(q["n_levels"]), int(q["level_cap"])
    c.clamp_p, c.serna_correct = int(q["clamp_p"]), int(q["serna_correct"])
    c.cand_cap = int(q.get("cand_cap", 4096))
    c.use_graph = int(q.get("use_graph", 1))
    for k in ("spacing", "h", "support", "block_edge", "rho0", "c0", "gamma", "visc_alpha",
              "visc_eps", "dt_base", "lambda_v", "lambda_f", "alpha_rts", "beta2", "beta_ratio"):
        setattr(c, k, float(q[k]))
    c.r_crit = float(q.get("r_crit", 0.0))
    for k in ("n_minor", "it_min", "it_max", "expand_layers", "local_fail", "global_limit",
              "short_majors", "two_ring_levels"):
        if k in q:
            setattr(c, k, int(q[k]))
    c.nbr_cap = int(q.get("nbr_cap", c.nbr_cap))
    for k in ("eta", "eta_T", "delta", "r_list", "pci_dt_min", "pci_dt_max", "pci_grow",
              "pci_shrink"):
        if k in q:
            setattr(c, k, float(q[k]))
    for k in ("pci_adapt_dt", "pci_grow_iters", "pci_shrink_iters", "phase_align"):
        if k in q:
            setattr(c, k, int(q[k]))
    c.mass = float(q.get("mass", 0.0))
    c.B = float(q.get("B", 0.0))
    for d in range(3):
        c.gravity[d] = float(q["gravity"][d])
        c.domain_min[d] = float(q["domain_min"][d])
        c.domain_max[d] = float(q["domain_max"][d])
    return c


def workspace_size(cfg: RtsConfig, n_fluid_max: int, n_wall_max: int) -> int:
    out = C.c_size_t(0)
    check(lib().rts_workspace_size(C.byref(cfg), int(n_fluid_max), int(n_wall_max), C.byref(out)))
    return int(out.value)


def create(cfg, n_fluid_max, n_wall_max, d_workspace, nbytes, stream):
    ctx = C.c_void_p()
    check(lib().rts_create(C.byref(cfg), int(n_fluid_max), int(n_wall_max), C.c_void_p(d_workspace),
                           int(nbytes), C.c_void_p(stream), C.byref(ctx)))
    return ctx


def create_batch(cfg, n_per_scene, n_wall_max, d_workspace, nbytes, stream):
    """A context of independent scenes of the given particle counts."""
    ctx = C.c_void_p()
    counts = (C.c_int64 * len(n_per_scene))(*[int(v) for v in n_per_scene])
    check(lib().rts_create_batch(C.byref(cfg), len(n_per_scene), counts, int(n_wall_max),
                                 C.c_void_p(d_workspace), int(nbytes), C.c_void_p(stream),
                                 C.byref(ctx)))
    return ctx


def init_dam_break(ctx, scene, first, counts, corner, spacing, jitter, seed, first_draw):
    c = (C.c_int32 * 3)(*[int(v) for v in counts])
    o = (C.c_double * 3)(*[float(v) for v in corner])
    check(lib().rts_init_dam_break(ctx, int(scene), int(first), c, o, float(spacing),
                                   float(jitter), int(seed), int(first_draw)), ctx)


def scene_stats(ctx, n_scenes):
    out = (RtsSceneStats * n_scenes)()
    check(lib().rts_get_scene_stats(ctx, out, int(n_scenes)), ctx)
    return [s.as_dict() for s in out]


def get_scene_state(ctx, scene, d_pos=0, d_vel=0, d_acc=0, d_rho=0, d_p=0, d_level=0):
    check(lib().rts_get_scene_state(ctx, int(scene), C.c_void_p(d_pos or None),
                                    C.c_void_p(d_vel or None), C.c_void_p(d_acc or None),
                                    C.c_void_p(d_rho or None), C.c_void_p(d_p or None),
                                    C.c_void_p(d_level or None)), ctx)


def create_static(cfg, n_fluid_max, n_wall_max, stream):
    """A context in the library's static device workspace (no allocation)."""
    ctx = C.c_void_p()
    check(lib().rts_create_static(C.byref(cfg), int(n_fluid_max), int(n_wall_max),
                                  C.c_void_p(stream), C.byref(ctx)))
    return ctx


def destroy(ctx):
    lib().rts_destroy(ctx)


def set_walls(ctx, d_pos, nw):
    check(lib().rts_set_walls(ctx, C.c_void_p(d_pos), int(nw)), ctx)


def set_state(ctx, d_pos, d_vel, n):
    check(lib().rts_set_state(ctx, C.c_void_p(d_pos), C.c_void_p(d_vel), int(n)), ctx)


def add_velocity(ctx, d_dv, n):
    check(lib().rts_add_velocity(ctx, C.c_void_p(d_dv), int(n)), ctx)


def assign_levels(ctx, n_levels):
    hist = (C.c_int32 * MAX_LEVELS)()
    check(lib().rts_assign_levels(ctx, hist), ctx)
    return list(hist)[:n_levels]


def advance(ctx, n_steps):
    check(lib().rts_advance(ctx, int(n_steps)), ctx)


def sync(ctx, raise_on_error=True):
    st = RtsStats()
    s = lib().rts_sync(ctx, C.byref(st))
    if raise_on_error:
        check(s, ctx)
    return st


def get_state(ctx, d_pos=0, d_vel=0, d_acc=0, d_rho=0, d_p=0, d_level=0):
    check(lib().rts_get_state(ctx, C.c_void_p(d_pos or None), C.c_void_p(d_vel or None),
                              C.c_void_p(d_acc or None), C.c_void_p(d_rho or None),
                              C.c_void_p(d_p or None), C.c_void_p(d_level or None)), ctx)


def state_bytes(ctx):
    out = C.c_size_t(0)
    check(lib().rts_state_bytes(ctx, C.byref(out)), ctx)
    return int(out.value)


def save_state(ctx, d_buf, cap):
    check(lib().rts_save_state(ctx, C.c_void_p(d_buf), int(cap)), ctx)


def load_state(ctx, d_buf, length):
    check(lib().rts_load_state(ctx, C.c_void_p(d_buf), int(length)), ctx)


def debug_get(ctx, what, d_out, cap_bytes):
    n = C.c_size_t(0)
    w = DBG[what] if isinstance(what, str) else int(what)
    check(lib().rts_debug_get(ctx, w, C.c_void_p(d_out), int(cap_bytes), C.byref(n)), ctx)
    return int(n.value)


def debug_count(ctx, what):
    """Element count of a debug view (a zero-capacity call reports it)."""
    n = C.c_size_t(0)
    w = DBG[what] if isinstance(what, str) else int(what)
    lib().rts_debug_get(ctx, w, C.c_void_p(1), 0, C.byref(n))
    return int(n.value)


def grid_info(ctx):
    nc = (C.c_int32 * 3)()
    nb = C.c_int64(0)
    m, B, dt = C.c_double(0), C.c_double(0), C.c_double(0)
    check(lib().rts_grid_info(ctx, nc, C.byref(nb), C.byref(m), C.byref(B), C.byref(dt)), ctx)
    return dict(nc=list(nc), nblocks=int(nb.value), mass=m.value, B=B.value, dt_base=dt.value)


def profile_advance(ctx, n_steps):
    """Per-kernel milliseconds summed over n_steps eager, event-bracketed steps."""
    ms = (C.c_double * len(PROF_KERNELS))()
    check(lib().rts_profile_advance(ctx, int(n_steps), ms), ctx)
    return dict(zip(PROF_KERNELS, list(ms)))


def autotune(ctx, steps, d_scratch, nbytes):
    t = RtsTune()
    check(lib().rts_autotune(ctx, int(steps), C.c_void_p(d_scratch), int(nbytes), C.byref(t)), ctx)
    return t.as_dict()


def get_tune(ctx):
    t = RtsTune()
    check(lib().rts_get_tune(ctx, C.byref(t)), ctx)
    return t.as_dict()


def set_tune(ctx, shape: dict):
    """Sets the launch shape from a dict like get_tune's (missing keys keep
    the current values)."""
    cur = get_tune(ctx)
    cur.update(shape)
    t = RtsTune()
    for k, _ in t._fields_:
        if k in cur:
            setattr(t, k, type(getattr(t, k))(cur[k]))
    check(lib().rts_set_tune(ctx, C.byref(t)), ctx)


def diff_desc(n_sub, ckpt_every, list_cap, dt, B, alpha):
    d = RtsDiffDesc()
    d.n_sub, d.ckpt_every, d.list_cap = int(n_sub), int(ckpt_every), int(list_cap)
    d.dt, d.B, d.alpha = float(dt), float(B), float(alpha)
    return d


def diff_tape_bytes(ctx, desc, n):
    out = C.c_size_t(0)
    check(lib().rts_diff_tape_bytes(ctx, C.byref(desc), int(n), C.byref(out)), ctx)
    return int(out.value)


def diff_forward(ctx, desc, n, d_x0, d_v0, d_xT, d_vT, d_tape, nbytes):
    check(lib().rts_diff_forward(ctx, C.byref(desc), int(n), C.c_void_p(d_x0), C.c_void_p(d_v0),
                                 C.c_void_p(d_xT), C.c_void_p(d_vT), C.c_void_p(d_tape),
                                 int(nbytes)), ctx)


def diff_backward(ctx, desc, n, d_xT_bar, d_vT_bar, d_x0_bar, d_v0_bar, d_tape, nbytes):
    gB, ga = C.c_double(0), C.c_double(0)
    check(lib().rts_diff_backward(ctx, C.byref(desc), int(n), C.c_void_p(d_xT_bar),
                                  C.c_void_p(d_vT_bar or None), C.c_void_p(d_x0_bar or None),
                                  C.c_void_p(d_v0_bar or None), C.byref(gB), C.byref(ga),
                                  C.c_void_p(d_tape), int(nbytes)), ctx)
    return gB.value, ga.value


def last_error(ctx):
    return lib().rts_last_error(ctx).decode()
