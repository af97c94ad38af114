"""Shared helpers of the GPU parity tests: oracle expectations computed from a
GPU snapshot (the arrays a base step started from)."""
from __future__ import annotations

import numpy as np

import oracle
from paper_2009_14514_amd.sim import decode_meta, neighbour_lists


def snapshot_after_step(sim):
    """Arrays of the last step: its input (previous order) and its outputs."""
    v = {"STEP": sim.sync().step - 1}       # base steps taken before the last one
    v.update({k: sim.debug(k) for k in (
        "PRE_POS", "PRE_VEL", "PRE_ACC", "PRE_META", "PRE_ID", "POS", "VEL", "ACC", "ACC_NEW",
        "META", "ID", "KEY", "PERM", "CELL_START", "BLK_LEVEL_RAW", "BLK_LEVEL", "NNB",
        "PRESSURE", "WALL_POS", "WALL_ID", "WALL_CELL_START")})
    return v


def expected_structure(cfg, snap):
    """Oracle keys / order / levels / flags for the step whose input is snap['PRE_*']."""
    info = oracle.derive(cfg)
    pre_pos = snap["PRE_POS"][:, :3]
    keys_old = oracle.keys(cfg, pre_pos)
    perm, start = oracle.sort(info.nblocks, keys_old)
    lraw = oracle.block_levels(cfg, keys_old, snap["PRE_VEL"][:, :3], snap["PRE_ACC"][:, :3])
    lvl = oracle.rmin(cfg, lraw)
    level0, _, age0, val0 = decode_meta(snap["PRE_META"])
    level1, val1, comp1 = oracle.flags(keys_old, lvl, level0, val0, step=snap["STEP"],
                                       phase_align=cfg.phase_align)
    age1 = np.where(comp1 == 1, 1, age0 + 1)
    return dict(keys=keys_old[perm], perm=perm, cell_start=start, lraw=lraw, lvl=lvl,
                level=level1[perm], validity=val1[perm], compute=comp1[perm], age=age1[perm],
                info=info)


def gpu_lists(sim, snap, rows):
    """GPU neighbour lists of the given sorted particles, as arrays."""
    lists, counts = neighbour_lists(sim)
    return [lists[i, :counts[i]].astype(np.uint32) for i in rows], counts


def oracle_lists(cfg, snap, want, cap=1024):
    pos_sorted = snap["PRE_POS"][snap["PERM"], :3]
    wpos = snap["WALL_POS"][:, :3]
    st, nbr, nnb = oracle.neighbors(cfg, pos_sorted, wpos, want=want, cap=cap)
    assert st == 0
    return nbr, nnb


def oracle_density(cfg, snap, which):
    x = snap["PRE_POS"][snap["PERM"], :3].astype(np.float64)
    w = snap["WALL_POS"][:, :3].astype(np.float64)
    return oracle.density(cfg, x, w, which=which)


def oracle_forces_stage(cfg, snap, which, term_sums=False):
    """Force stage alone: the oracle consumes the GPU's own float density and
    pressure of every particle (fresh for active, stale for the others).
    With ``term_sums`` also each particle's sum of term magnitudes."""
    perm = snap["PERM"]
    x = snap["PRE_POS"][perm, :3].astype(np.float64)
    v = snap["PRE_VEL"][perm, :3].astype(np.float64)
    rho = snap["POS"][:, 3].astype(np.float64)
    p = snap["VEL"][:, 3].astype(np.float64) * rho * rho   # the GPU keeps p / rho^2
    w = snap["WALL_POS"][:, :3].astype(np.float64)
    return oracle.forces(cfg, x, v, rho, p, w, which=which, term_sums=term_sums)
