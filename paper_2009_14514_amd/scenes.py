"""Seeded synthetic scene generators (dam-break columns, box walls, batches).

This module only places particles and names run parameters.  It holds none
of the method's arithmetic: no kernel, no mass calibration, no time-step
criterion.  Both the HIP library (through the Python binding) and the CPU
oracle consume the arrays it returns, so the two sides start from identical
inputs.

Random draws use SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): output k of the stream with
seed S is mix(S + (k + 1) * 0x9E3779B97F4A7C15).  The jitter of particle i
along axis c uses output k = 3 i + c, u = (out >> 40) * 2^-24, and the offset
is j * (2u - 1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, idx: np.ndarray) -> np.ndarray:
    """Outputs number ``idx`` (0-based, uint64 array) of the SplitMix64 stream."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (idx.astype(np.uint64) + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform01(seed: int, idx: np.ndarray) -> np.ndarray:
    """24-bit uniform in [0, 1) from stream outputs ``idx``."""
    return (splitmix64(seed, idx) >> np.uint64(40)).astype(np.float64) * (2.0 ** -24)


def lattice_column(counts, spacing, corner, jitter=0.0, seed=0, first_index=0):
    """Particles at corner + (i + 1/2) * spacing, i over ``counts`` (x fastest).

    Returns float64 (N, 3).  ``jitter`` is the half-width of the uniform
    per-axis offset; ``first_index`` offsets the SplitMix64 stream so that
    several columns of one scene draw disjoint numbers.
    """
    nx, ny, nz = (int(c) for c in counts)
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    idx = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    pos = np.asarray(corner, np.float64)[None, :] + (idx + 0.5) * spacing
    if jitter != 0.0 and pos.shape[0] > 0:
        k = np.arange(pos.shape[0] * 3, dtype=np.uint64) + np.uint64(3 * first_index)
        u = uniform01(seed, k).reshape(-1, 3)
        pos = pos + jitter * (2.0 * u - 1.0)
    return pos


def box_walls(box_min, box_max, spacing, layers):
    """Static wall particles: a shell ``layers`` deep around the box.

    Lattice points at box_min + (i + 1/2) * spacing for i in [-layers, n + layers)
    per axis, minus the points inside the box.  Returns float64 (Nw, 3).
    """
    bmin = np.asarray(box_min, np.float64)
    bmax = np.asarray(box_max, np.float64)
    n = np.rint((bmax - bmin) / spacing).astype(np.int64)
    axes = [np.arange(-layers, n[c] + layers) for c in range(3)]
    iz, iy, ix = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    inside = (ix >= 0) & (ix < n[0]) & (iy >= 0) & (iy < n[1]) & (iz >= 0) & (iz < n[2])
    keep = ~inside
    idx = np.stack([ix[keep], iy[keep], iz[keep]], axis=1).astype(np.float64)
    return bmin[None, :] + (idx + 0.5) * spacing


@dataclass
class Scene:
    """One scene: fluid and wall particles plus the run parameters."""
    name: str
    pos: np.ndarray                      # (N, 3) float64, fluid
    vel: np.ndarray                      # (N, 3) float64
    walls: np.ndarray                    # (Nw, 3) float64
    params: dict = field(default_factory=dict)
    # batched scenes: fluid index range (start, end) and placement offset of
    # each sub-scene, and the sub-scenes as they run on their own
    parts: list = field(default_factory=list)
    offsets: list = field(default_factory=list)
    subscenes: list = field(default_factory=list)
    # the lattice columns the fluid was generated from (scene, first particle
    # in the scene, counts, corner, spacing, jitter, seed, first draw), so a
    # batched context can generate them on the device instead
    columns: list = field(default_factory=list)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @property
    def nw(self) -> int:
        return int(self.walls.shape[0])


def base_params(spacing, box_min, box_max, *, c0, layers=4, h_ratio=2.0,
                support_ratio=2.0, edge_ratio=1.0, dt_base=0.0, level_cap=3,
                n_levels=4, mode="rts", solver="wcsph"):
    """Parameter dictionary shared by both sides.

    ``dt_base = 0`` asks each side to take the base step from the sound-speed
    criterion.  The domain is the box grown by the wall shell.
    """
    h = h_ratio * spacing
    support = support_ratio * h
    margin = layers * spacing
    return dict(
        solver=solver, mode=mode,
        spacing=spacing, h=h, support=support, block_edge=edge_ratio * support,
        rho0=1000.0, c0=float(c0), gamma=7.0, visc_alpha=0.05, visc_eps=0.01,
        gravity=(0.0, -9.81, 0.0),
        box_min=tuple(float(b) for b in box_min), box_max=tuple(float(b) for b in box_max),
        domain_min=tuple(float(b) - margin for b in box_min),
        domain_max=tuple(float(b) + margin for b in box_max),
        dt_base=float(dt_base), r_crit=2.0 * spacing, lambda_v=0.4, lambda_f=0.25,
        alpha_rts=0.4 if solver == "wcsph" else 1.0, beta2=0.4, beta_ratio=0.2,
        n_levels=n_levels, level_cap=level_cap, clamp_p=1, serna_correct=1,
        # WCSPH: a particle taking level l is due at the next multiple of 2^l
        phase_align=1,
        wall_layers=layers,
        # PCISPH settings (unused by WCSPH)
        eta=0.01, eta_T=0.0025, it_min=3, it_max=50, n_minor=4, expand_layers=4,
        local_fail=3, global_limit=6, short_majors=10, delta=0.0, r_list=0.0,
        nbr_cap=512,
    )


def sound_speed_for_column(height, g=9.81, factor=20.0):
    """c0 = factor * sqrt(2 g H) for a column of height H.

    sqrt(2 g H) bounds the collapse speed; weakly compressible SPH takes c0 at
    least ten times the flow speed.  Twenty times keeps the maximum
    compression of the 250,000-particle dam break below 1 % over its first
    500 base steps for both regional and global stepping (ten times does not).
    """
    return factor * math.sqrt(2.0 * g * height)


def dam_break_small(seed=0):
    """4,096 particles (16^3, spacing 0.02 m) in a 0.6 x 0.4 x 0.4 m box, c0 = 20 m/s,
    global fixed dt = 2e-4 s, jitter +-1e-4 m."""
    s = 0.02
    bmin, bmax = (0.0, 0.0, 0.0), (0.6, 0.4, 0.4)
    pos = lattice_column((16, 16, 16), s, bmin, jitter=1e-4, seed=seed)
    p = base_params(s, bmin, bmax, c0=20.0, dt_base=2e-4, level_cap=0, mode="global_fixed")
    return Scene("dam_break_4k", pos, np.zeros_like(pos), box_walls(bmin, bmax, s, p["wall_layers"]), p)


def dam_break_column(counts=(50, 100, 50), spacing=0.01, box=(2.0, 1.0, 1.0), seed=0,
                     jitter_frac=0.005, c0=None, mode="rts", level_cap=3, name=None):
    """Dam break: a column of ``counts`` lattice particles at the x = 0 corner of a box.

    The default is the 250,000-particle column (0.5 x 1.0 x 0.5 m, spacing 0.01 m)
    in a 2 x 1 x 1 m box with block levels 0..3.
    """
    bmin, bmax = (0.0, 0.0, 0.0), tuple(float(b) for b in box)
    height = counts[1] * spacing
    if c0 is None:
        c0 = sound_speed_for_column(height)
    pos = lattice_column(counts, spacing, bmin, jitter=jitter_frac * spacing, seed=seed)
    p = base_params(spacing, bmin, bmax, c0=c0, dt_base=0.0, level_cap=level_cap, mode=mode)
    p["column_height"] = height
    return Scene(name or f"dam_break_{pos.shape[0]}", pos, np.zeros_like(pos),
                 box_walls(bmin, bmax, spacing, p["wall_layers"]), p)


def pcisph_params(spacing, bmin, bmax, height, dt_base, mode="rts"):
    """PCISPH runs take the paper's kernel support r = 2s (h = s) on a grid of
    block edge 1.1 r = 2.2s, with two wall layers.  (At support 4s the
    standard prototype-neighbourhood delta over-corrects and the iteration
    diverges.)  c0 only scales the artificial viscosity."""
    p = base_params(spacing, bmin, bmax, c0=sound_speed_for_column(height), layers=2,
                    h_ratio=1.0, support_ratio=2.0, edge_ratio=1.1, dt_base=dt_base,
                    solver="pcisph", level_cap=3, mode=mode)
    p["nbr_cap"] = 128      # about 45 neighbours within 2.2s at rest
    return p


def double_dam_break(spacing=0.4 / 63, col=(0.4, 0.8, 0.4), box=(2.0, 1.0, 1.0), seed=0,
                     jitter_frac=0.005, dt_base=5e-4):
    """PCISPH double dam break: two columns at both x-ends of a 2 x 1 x 1 m box.

    At spacing 0.4/63 m each column is 63 x 126 x 63 (1,000,188 particles total).
    The base step is 5e-4 s: at 1e-3 s standard PCISPH itself diverges at
    this spacing within 0.1 s (the column sinks into the two-layer floor),
    while 5e-4 s keeps both standard and regional PCISPH below 1 %.
    """
    n = tuple(int(round(c / spacing)) for c in col)
    bmin, bmax = (0.0, 0.0, 0.0), tuple(float(b) for b in box)
    a = lattice_column(n, spacing, (0.0, 0.0, 0.0), jitter=jitter_frac * spacing, seed=seed)
    b = lattice_column(n, spacing, (box[0] - n[0] * spacing, 0.0, 0.0),
                       jitter=jitter_frac * spacing, seed=seed, first_index=a.shape[0])
    pos = np.concatenate([a, b], axis=0)
    p = pcisph_params(spacing, bmin, bmax, col[1], dt_base)
    return Scene(f"double_dam_break_{pos.shape[0]}", pos, np.zeros_like(pos),
                 box_walls(bmin, bmax, spacing, p["wall_layers"]), p)


def pcisph_dam_break_small(counts=(10, 20, 10), spacing=0.02, box=(0.8, 0.5, 0.3), seed=0,
                           dt_base=1e-3, mode="rts", v0=0.0):
    """Small PCISPH double dam break: two ``counts`` columns at both x-ends of
    the box (4,000 particles by default), thrown at each other with speed
    ``v0`` (m/s) along x."""
    bmin, bmax = (0.0, 0.0, 0.0), tuple(float(b) for b in box)
    a = lattice_column(counts, spacing, (0.0, 0.0, 0.0), jitter=0.005 * spacing, seed=seed)
    b = lattice_column(counts, spacing, (box[0] - counts[0] * spacing, 0.0, 0.0),
                       jitter=0.005 * spacing, seed=seed, first_index=a.shape[0])
    pos = np.concatenate([a, b], axis=0)
    vel = np.zeros_like(pos)
    vel[: a.shape[0], 0] = v0
    vel[a.shape[0]:, 0] = -v0
    p = pcisph_params(spacing, bmin, bmax, counts[1] * spacing, dt_base, mode)
    return Scene(f"pcisph_double_dam_break_{pos.shape[0]}", pos, vel,
                 box_walls(bmin, bmax, spacing, p["wall_layers"]), p)


def pcisph_thrown_columns(speeds=(0.0, 0.5, 1.5, 12.0), counts=(6, 6, 6), spacing=0.02,
                          box=(1.6, 0.7, 0.3), seed=0, dt_base=1e-3, mode="rts", wall_gap=0.25):
    """Four PCISPH columns that start in four different regions (paper's
    Eq. 2-3 at the default thresholds and a base step of 1e-3 s: 0 m/s
    region 4, 0.5 m/s region 3, 1.5 m/s region 2, 12 m/s region 1):

      A at rest on the floor at the left wall;
      B on the floor, thrown towards +x at speeds[1];
      C on the floor, thrown towards the right wall at speeds[2],
        ``wall_gap`` spacings from it (by default a quarter spacing, so that
        it hits the wall within a few minor steps: local and extra global
        iterations, an early end of a major step);
      D in the air above B and C, thrown towards -x at speeds[3].

    The columns are at least 6 blocks (of edge 2.2 spacings) apart, more
    than the 4-block growth of regions 1 and 2, so the four regions coexist.
    """
    bmin, bmax = (0.0, 0.0, 0.0), tuple(float(b) for b in box)
    w = counts[0] * spacing
    corners = [(0.0, 0.0, 0.0), (0.5, 0.0, 0.0), (box[0] - w - wall_gap * spacing, 0.0, 0.0),
               (0.9, 0.45, 0.0)]
    dirs = [(0.0, 0.0, 0.0), (1.0, 0.0, 0.0), (1.0, 0.0, 0.0), (-1.0, 0.0, 0.0)]
    pos_all, vel_all = [], []
    first = 0
    for corner, d, v in zip(corners, dirs, speeds):
        p = lattice_column(counts, spacing, corner, jitter=0.005 * spacing, seed=seed,
                           first_index=first)
        first += p.shape[0]
        pos_all.append(p)
        vel_all.append(np.tile(np.asarray(d) * float(v), (p.shape[0], 1)))
    pos = np.concatenate(pos_all, axis=0)
    vel = np.concatenate(vel_all, axis=0)
    p = pcisph_params(spacing, bmin, bmax, counts[1] * spacing, dt_base, mode)
    return Scene(f"pcisph_thrown_columns_{pos.shape[0]}", pos, vel,
                 box_walls(bmin, bmax, spacing, p["wall_layers"]), p)


def pcisph_column(counts=(8, 12, 8), spacing=0.02, box=(0.16, 0.5, 0.16), seed=0,
                  dt_base=1e-3, mode="rts"):
    """One PCISPH column at the x = 0 corner of the box."""
    bmin, bmax = (0.0, 0.0, 0.0), tuple(float(b) for b in box)
    pos = lattice_column(counts, spacing, bmin, jitter=0.005 * spacing, seed=seed)
    p = pcisph_params(spacing, bmin, bmax, counts[1] * spacing, dt_base, mode)
    return Scene(f"pcisph_column_{pos.shape[0]}", pos, np.zeros_like(pos),
                 box_walls(bmin, bmax, spacing, p["wall_layers"]), p)


def batch_sizes(n_scenes=64, lo=2000, hi=200000, seed=0):
    """Particle counts log-uniform in [lo, hi] and column aspect ratios U(0.3, 1.5)."""
    k = np.arange(2 * n_scenes, dtype=np.uint64)
    u = uniform01(seed, k).reshape(n_scenes, 2)
    counts = np.rint(np.exp(math.log(lo) + u[:, 0] * (math.log(hi) - math.log(lo)))).astype(np.int64)
    aspect = 0.3 + 1.2 * u[:, 1]
    return counts, aspect


def batched_dam_breaks(n_scenes=64, lo=2000, hi=200000, seed=0, spacing=0.01,
                       box=(2.0, 1.0, 1.0), counts=None):
    """Independent dam-break scenes of uneven size in one particle set.

    Scene k is a column of about N_k particles (log-uniform in [lo, hi]) with
    aspect ratio a_k (height / width, U(0.3, 1.5)): n_x = n_z =
    round((N_k / a_k)^(1/3)), n_y = round(a_k n_x), at the x = 0 corner of
    its own box.  The boxes (with their wall shells) are tiled in space far
    enough apart that no particle of one scene is within the kernel support
    of another scene's particles, so one step of the whole set advances every
    scene independently.  All scenes share the sound speed of the tallest
    column and hence the base step.  ``counts`` may give (n_x, n_y, n_z) per
    scene directly.
    """
    if counts is None:
        n_k, a_k = batch_sizes(n_scenes, lo, hi, seed)
        counts = []
        for n, a in zip(n_k, a_k):
            nx = max(int(round((n / a) ** (1.0 / 3.0))), 1)
            ny = max(int(round(a * nx)), 1)
            nx = min(nx, int(box[0] / spacing))
            ny = min(ny, int(box[1] / spacing))
            nz = min(nx, int(box[2] / spacing))
            counts.append((nx, ny, nz))
    counts = [tuple(int(c) for c in cc) for cc in counts]
    for cc in counts:
        if any(cc[d] * spacing > box[d] + 1e-12 for d in range(3)):
            raise ValueError(f"column {cc} does not fit the box {box}")
    n_scenes = len(counts)
    layers = 4
    margin = layers * spacing
    gap = 4.0 * spacing                       # at least one block edge between wall shells
    pitch = np.array([box[0], box[1], box[2]]) + 2.0 * margin + gap
    per_row = int(math.ceil(n_scenes ** (1.0 / 3.0)))
    height = max(c[1] for c in counts) * spacing
    pos_all, wall_all, parts, offsets, subs = [], [], [], [], []
    start = 0
    walls0 = box_walls((0.0, 0.0, 0.0), box, spacing, layers)
    c0 = sound_speed_for_column(height)
    columns = []
    for k, cc in enumerate(counts):
        off = pitch * np.array([k % per_row, (k // per_row) % per_row, k // (per_row * per_row)])
        local = lattice_column(cc, spacing, (0.0, 0.0, 0.0), jitter=0.005 * spacing, seed=seed + k)
        # the column generated in place (the same lattice and draws, rounded
        # at its own position), as rts_init_dam_break produces it
        pos = lattice_column(cc, spacing, off, jitter=0.005 * spacing, seed=seed + k)
        columns.append(dict(scene=k, first=0, counts=cc, corner=tuple(float(o) for o in off),
                            spacing=spacing, jitter=0.005 * spacing, seed=seed + k,
                            first_draw=0))
        pos_all.append(pos)
        wall_all.append(walls0 + off[None, :])
        parts.append((start, start + pos.shape[0]))
        offsets.append(tuple(float(o) for o in off))
        subs.append(Scene(f"batch_part_{k}", local, np.zeros_like(local), walls0,
                          base_params(spacing, (0.0, 0.0, 0.0), box, c0=c0, dt_base=0.0,
                                      level_cap=3)))
        start += pos.shape[0]
    pos = np.concatenate(pos_all, axis=0)
    walls = np.concatenate(wall_all, axis=0)
    top = pitch * np.array([min(n_scenes, per_row) - 1,
                            min((n_scenes - 1) // per_row, per_row - 1),
                            (n_scenes - 1) // (per_row * per_row)])
    bmax = tuple(float(t + b) for t, b in zip(top, box))
    p = base_params(spacing, (0.0, 0.0, 0.0), bmax, c0=c0, dt_base=0.0, level_cap=3)
    return Scene(f"batched_{n_scenes}_scenes_{pos.shape[0]}", pos, np.zeros_like(pos), walls, p,
                 parts=parts, offsets=offsets, subscenes=subs, columns=columns)


def normal01(seed: int, idx: np.ndarray) -> np.ndarray:
    """Standard normal draws by Box-Muller on pairs of SplitMix64 outputs
    (2k, 2k + 1) of the stream."""
    idx = np.asarray(idx, np.uint64)
    u1 = uniform01(seed, 2 * idx)
    u2 = uniform01(seed, 2 * idx + np.uint64(1))
    u1 = np.maximum(u1, 2.0 ** -25)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def diff_scene(counts=(8, 8, 8), spacing=0.01, box=(0.3, 0.3, 0.3), seed=0, v_scale=0.2,
               dt=1e-4, n_sub=16, target_sigma=0.005):
    """Differentiable dam break: a column with seeded initial velocities
    U(-v_scale, v_scale) per component; run for n_sub substeps of dt.  The
    target of the loss is the nominal final positions plus N(0, sigma^2) per
    coordinate (drawn from stream seed + 1 over index 3 i + c); it is
    produced by the caller from its own nominal run."""
    bmin = (0.0, 0.0, 0.0)
    pos = lattice_column(counts, spacing, bmin, jitter=0.005 * spacing, seed=seed)
    k = np.arange(pos.shape[0] * 3, dtype=np.uint64) + np.uint64(1 << 40)
    vel = (v_scale * (2.0 * uniform01(seed, k) - 1.0)).reshape(-1, 3)
    height = max(counts[1] * spacing, 0.5)
    p = base_params(spacing, bmin, box, c0=sound_speed_for_column(height), dt_base=dt,
                    level_cap=0, mode="global_fixed")
    p.update(diff_dt=dt, diff_substeps=n_sub, target_sigma=target_sigma, clamp_p=0)
    return Scene(f"diff_dam_break_{pos.shape[0]}", pos, vel,
                 box_walls(bmin, box, spacing, p["wall_layers"]), p)


def target_noise(n, sigma=0.005, seed=0):
    """N(0, sigma^2) offsets per coordinate for the loss target."""
    return sigma * normal01(seed + 1, np.arange(3 * n, dtype=np.uint64)).reshape(n, 3)


def wcsph_double_dam_break(counts=(40, 80, 40), spacing=0.01, box=(2.0, 1.0, 1.0), seed=0,
                           mode="rts"):
    """WCSPH double dam break: two columns at both x-ends of the box (the
    paper's double dam break, here 256,000 particles at spacing 0.01 m).
    The sound speed is taken for the box height, not the column's: where the
    two fronts collide the compression exceeds a single collapse's (1.06 %
    within 500 base steps at 20 sqrt(2 g 0.8))."""
    bmin, bmax = (0.0, 0.0, 0.0), tuple(float(b) for b in box)
    a = lattice_column(counts, spacing, (0.0, 0.0, 0.0), jitter=0.005 * spacing, seed=seed)
    b = lattice_column(counts, spacing, (box[0] - counts[0] * spacing, 0.0, 0.0),
                       jitter=0.005 * spacing, seed=seed, first_index=a.shape[0])
    pos = np.concatenate([a, b], axis=0)
    p = base_params(spacing, bmin, bmax, c0=sound_speed_for_column(box[1]), dt_base=0.0,
                    level_cap=3, mode=mode)
    return Scene(f"wcsph_double_dam_break_{pos.shape[0]}", pos, np.zeros_like(pos),
                 box_walls(bmin, bmax, spacing, p["wall_layers"]), p)


def block_drop(column=(50, 60, 50), block=(30, 30, 30), spacing=0.01, box=(2.0, 1.0, 1.0),
               drop_at=(1.0, 0.65, 0.2), seed=0, mode="rts"):
    """Dam break with a second block of liquid released above the floor at
    the same moment (the paper's block-drop scene, here 177,000 particles)."""
    bmin, bmax = (0.0, 0.0, 0.0), tuple(float(b) for b in box)
    a = lattice_column(column, spacing, (0.0, 0.0, 0.0), jitter=0.005 * spacing, seed=seed)
    b = lattice_column(block, spacing, drop_at, jitter=0.005 * spacing, seed=seed,
                       first_index=a.shape[0])
    pos = np.concatenate([a, b], axis=0)
    top = drop_at[1] + block[1] * spacing
    p = base_params(spacing, bmin, bmax, c0=sound_speed_for_column(top), dt_base=0.0,
                    level_cap=3, mode=mode)
    return Scene(f"block_drop_{pos.shape[0]}", pos, np.zeros_like(pos),
                 box_walls(bmin, bmax, spacing, p["wall_layers"]), p)
