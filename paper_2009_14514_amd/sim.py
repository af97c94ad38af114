"""Python front end of the RTS library: torch supplies device memory and the
stream, librts.so does every step of the simulation.
"""
from __future__ import annotations

import numpy as np

from . import _rts


def _torch():
    import torch
    return torch


def _planes(a: np.ndarray) -> np.ndarray:
    """(N, 3) -> contiguous float32 planes x[N], y[N], z[N]."""
    a = np.asarray(a, dtype=np.float32).reshape(-1, 3)
    return np.ascontiguousarray(a.T).reshape(-1)


def _from_planes(a: np.ndarray, n: int) -> np.ndarray:
    return np.asarray(a, dtype=np.float32).reshape(3, n).T.copy()


def _aligned(buf, align=256):
    addr = buf.data_ptr()
    return addr + (-addr) % align


class Simulation:
    """One scene simulated by the HIP library.

    ``scene`` is a :class:`paper_2009_14514_amd.scenes.Scene`; keyword
    arguments override entries of its parameter dictionary.
    ``static_workspace`` places the context in the library's static device
    workspace (rts_create_static) instead of a torch allocation.  A scene
    with ``parts`` (independent sub-scenes) gets a batched context
    (rts_create_batch); with ``device_init`` its lattice columns are
    generated on the device (rts_init_dam_break) instead of uploaded.
    """

    def __init__(self, scene, device="cuda", n_fluid_max=None, n_wall_max=None,
                 static_workspace=False, device_init=False, **over):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("the RTS library needs a GPU; none is visible")
        _rts.lib()  # fails loudly if librts.so is missing
        self.params = dict(scene.params)
        self.params.update(over)
        self.cfg = _rts.config_from_params(self.params)
        self.device = torch.device(device)
        self.n = scene.n
        self.nw = scene.nw
        self.n_fluid_max = int(n_fluid_max if n_fluid_max is not None else max(self.n, 1))
        self.n_wall_max = int(n_wall_max if n_wall_max is not None else max(self.nw, 1))
        self.stream = torch.cuda.current_stream(self.device)
        self.n_scenes = max(len(scene.parts), 1)
        if scene.parts and not static_workspace:
            counts = [int(b - a) for a, b in scene.parts]
            nbytes = _rts.workspace_size(self.cfg, sum(counts), self.n_wall_max)
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            self.ctx = _rts.create_batch(self.cfg, counts, self.n_wall_max,
                                         _aligned(self.workspace), nbytes, self.stream.cuda_stream)
        elif static_workspace:
            # the library's own device array: nothing is allocated here
            self.workspace = None
            self.ctx = _rts.create_static(self.cfg, self.n_fluid_max, self.n_wall_max,
                                          self.stream.cuda_stream)
        else:
            nbytes = _rts.workspace_size(self.cfg, self.n_fluid_max, self.n_wall_max)
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            self.ctx = _rts.create(self.cfg, self.n_fluid_max, self.n_wall_max,
                                   _aligned(self.workspace), nbytes, self.stream.cuda_stream)
        self.info = _rts.grid_info(self.ctx)
        self.set_walls(scene.walls)
        if device_init:
            if not scene.columns:
                raise ValueError("the scene records no lattice columns to generate")
            self.init_columns(scene.columns)
        else:
            self.set_state(scene.pos, scene.vel)

    # -- state ------------------------------------------------------------
    def _dev(self, host: np.ndarray):
        torch = _torch()
        return torch.from_numpy(np.ascontiguousarray(host)).to(self.device)

    def set_walls(self, walls):
        walls = np.asarray(walls).reshape(-1, 3)
        self.nw = walls.shape[0]
        t = self._dev(_planes(walls)) if self.nw else None
        _rts.set_walls(self.ctx, t.data_ptr() if t is not None else 0, self.nw)
        self._keep_walls = t
        self.stream.synchronize()

    def set_state(self, pos, vel=None):
        pos = np.asarray(pos).reshape(-1, 3)
        self.n = pos.shape[0]
        tp = self._dev(_planes(pos)) if self.n else None
        tv = self._dev(_planes(vel)) if (self.n and vel is not None) else None
        _rts.set_state(self.ctx, tp.data_ptr() if tp is not None else 0,
                       tv.data_ptr() if tv is not None else 0, self.n)
        self.stream.synchronize()

    def add_velocity(self, dv):
        """Adds a velocity change (N, 3) in caller order, keeping levels and flags."""
        t = self._dev(_planes(dv))
        _rts.add_velocity(self.ctx, t.data_ptr(), self.n)
        self.stream.synchronize()

    def init_columns(self, columns):
        """Generates lattice columns on the device (rts_init_dam_break); each
        column is a dict of scene, first, counts, corner, spacing, jitter,
        seed, first_draw."""
        for c in columns:
            _rts.init_dam_break(self.ctx, c["scene"], c["first"], c["counts"], c["corner"],
                                c["spacing"], c["jitter"], c["seed"], c["first_draw"])
        self.stream.synchronize()

    def scene_stats(self):
        """Per-scene counters of the last step (rts_get_scene_stats)."""
        return _rts.scene_stats(self.ctx, self.n_scenes)

    def scene_state(self, k):
        """Positions, velocities, density, pressure and level of scene k's
        particles, in their caller order within the scene."""
        torch = _torch()
        st = self.scene_stats()[k]
        n = int(st["n"])
        buf = torch.zeros(max(n, 1) * 8, dtype=torch.float32, device=self.device)
        lev = torch.zeros(max(n, 1), dtype=torch.uint8, device=self.device)
        base = buf.data_ptr()
        _rts.get_scene_state(self.ctx, k, base, base + 12 * n, 0, base + 24 * n,
                             base + 28 * n, lev.data_ptr())
        self.stream.synchronize()
        h = buf.cpu().numpy()
        return dict(pos=_from_planes(h[:3 * n], n), vel=_from_planes(h[3 * n:6 * n], n),
                    rho=h[6 * n:7 * n].copy(), p=h[7 * n:8 * n].copy(),
                    level=lev.cpu().numpy()[:n].copy())

    def advance(self, n_steps=1):
        _rts.advance(self.ctx, n_steps)

    def profile(self, n_steps):
        return _rts.profile_advance(self.ctx, n_steps)

    def sync(self, raise_on_error=True):
        return _rts.sync(self.ctx, raise_on_error)

    def assign_levels(self):
        return _rts.assign_levels(self.ctx, self.cfg.n_levels)

    def state(self):
        """Positions, velocities, accelerations, density, pressure, level in caller order."""
        torch = _torch()
        n = self.n
        buf = torch.zeros(max(3 * n, 1) * 3 + 2 * max(n, 1), dtype=torch.float32, device=self.device)
        lev = torch.zeros(max(n, 1), dtype=torch.uint8, device=self.device)
        base = buf.data_ptr()
        o = [0, 3 * n, 6 * n, 9 * n, 10 * n]
        _rts.get_state(self.ctx, base + 4 * o[0], base + 4 * o[1], base + 4 * o[2],
                       base + 4 * o[3], base + 4 * o[4], lev.data_ptr())
        self.stream.synchronize()
        h = buf.cpu().numpy()
        return dict(pos=_from_planes(h[o[0]:o[1]], n), vel=_from_planes(h[o[1]:o[2]], n),
                    acc=_from_planes(h[o[2]:o[3]], n), rho=h[o[3]:o[4]].copy(),
                    p=h[o[4]:o[4] + n].copy(), level=lev.cpu().numpy()[:n].copy())

    def autotune(self, steps=10):
        """Times the candidate launch shapes on the current state and keeps the
        fastest (the state is restored afterwards)."""
        torch = _torch()
        nb = _rts.state_bytes(self.ctx)
        scratch = torch.empty(nb, dtype=torch.uint8, device=self.device)
        return _rts.autotune(self.ctx, steps, scratch.data_ptr(), nb)

    def tune(self):
        return _rts.get_tune(self.ctx)

    def set_tune(self, **shape):
        """Sets launch-shape fields (grid_wave, grid_search, grid_force,
        search_threads, force_lanes); no shape changes any result."""
        _rts.set_tune(self.ctx, shape)

    def save(self):
        torch = _torch()
        nb = _rts.state_bytes(self.ctx)
        buf = torch.empty(nb, dtype=torch.uint8, device=self.device)
        _rts.save_state(self.ctx, buf.data_ptr(), nb)
        return buf

    def load(self, buf):
        _rts.load_state(self.ctx, buf.data_ptr(), buf.numel())
        self.stream.synchronize()

    # -- debug views --------------------------------------------------------
    _VIEW = {
        "POS": (np.float32, 4), "VEL": (np.float32, 4), "ACC": (np.float32, 4),
        "ACC_NEW": (np.float32, 4), "META": (np.uint32, 1), "ID": (np.uint32, 1),
        "KEY": (np.uint32, 1), "PERM": (np.uint32, 1), "CELL_START": (np.uint32, 1),
        "BLK_LEVEL_RAW": (np.uint8, 1), "BLK_LEVEL": (np.uint8, 1), "NNB": (np.uint32, 1),
        "NBR": (np.uint32, 1), "PRESSURE": (np.float32, 1), "PRE_POS": (np.float32, 4),
        "PRE_VEL": (np.float32, 4), "PRE_ACC": (np.float32, 4), "PRE_META": (np.uint32, 1),
        "PRE_ID": (np.uint32, 1), "WALL_POS": (np.float32, 4), "WALL_ID": (np.uint32, 1),
        "WALL_CELL_START": (np.uint32, 1), "OCCUPIED": (np.uint32, 1),
        "BLK_STATS": (np.uint32, 4),
        "PCI_XS": (np.float32, 4), "PCI_PV": (np.float32, 4), "PCI_FVG": (np.float32, 4),
        "PCI_FP": (np.float32, 4), "PCI_SE": (np.uint8, 1), "PCI_OB": (np.uint8, 1),
        "PCI_DILATED": (np.uint8, 1), "PCI_LISTS": (np.uint32, 1),
    }

    def debug(self, what: str) -> np.ndarray:
        torch = _torch()
        dt, width = self._VIEW[what]
        count = _rts.debug_count(self.ctx, what)
        esz = np.dtype(dt).itemsize * width
        buf = torch.zeros(max(count * esz, 1), dtype=torch.uint8, device=self.device)
        _rts.debug_get(self.ctx, what, buf.data_ptr(), buf.numel())
        self.stream.synchronize()
        out = buf.cpu().numpy()[: count * esz].view(dt)
        return out.reshape(-1, width) if width > 1 else out

    def close(self):
        if getattr(self, "ctx", None):
            self.stream.synchronize()
            _rts.destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def neighbour_lists(sim):
    """Canonical lists of the last step's active particles: (rows (n, width), counts)."""
    raw = sim.debug("NBR")
    n, w = sim.n, _rts.DEBUG_NBR_ROW
    return raw[: n * w].reshape(n, w), raw[n * w: n * w + n]


def pcisph_lists(sim):
    """PCISPH neighbour lists: (rows (n, nbr_cap), counts)."""
    raw = sim.debug("PCI_LISTS")
    n, w = sim.n, int(sim.cfg.nbr_cap)
    return raw[: n * w].reshape(n, w), raw[n * w: n * w + n]


def decode_meta(m: np.ndarray):
    """Splits meta words into (level, compute, age, validity)."""
    m = np.asarray(m, np.uint32)
    level = (m & 0xF).astype(np.int32)
    compute = ((m >> 4) & 1).astype(np.uint8)
    age = ((m >> 5) & 0x7FF).astype(np.int32)
    validity = (m >> 16).astype(np.uint16).view(np.int16).astype(np.int32)
    return level, compute, age, validity
