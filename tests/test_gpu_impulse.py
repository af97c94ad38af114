"""Pre-emption after an external impulse, GPU against the oracle.

Section 4.2 (pre-emption) and Algorithm 1: a particle takes its block's
level again when its validity runs out or when its block's level differs
from its own, so a block whose particles are suddenly fast drops to a
smaller step at the next base step, R_min takes its occupied neighbours
down with it, and their particles that were in the middle of a longer step
recompute at once.  The impulse enters through rts_add_velocity, which
changes velocities and nothing else; the oracle gets the same change.
"""
import numpy as np
import pytest

import oracle
from paper_2009_14514_amd import scenes
from paper_2009_14514_amd.sim import Simulation, decode_meta

from parity import snapshot_after_step
from test_gpu_wcsph import TRAJ_TOL, check_structure, developed, f32, rts_scene

pytestmark = pytest.mark.gpu


def ring_of(key, nc):
    bx, rest = key % nc[0], key // nc[0]
    by, bz = rest % nc[1], rest // nc[1]
    out = []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                x, y, z = bx + dx, by + dy, bz + dz
                if 0 <= x < nc[0] and 0 <= y < nc[1] and 0 <= z < nc[2]:
                    out.append(x + nc[0] * (y + nc[1] * z))
    return np.array(out)


def test_impulse_preempts_its_block_and_the_ring_around_it():
    sc = developed(rts_scene())
    sim = Simulation(sc)
    ref = oracle.WCSPH(sc.params, f32(sc.pos), vel=f32(sc.vel), walls=f32(sc.walls))
    sim.advance(6)
    sim.sync()
    ref.step(6)
    cfg = oracle.cfg_from_params(sc.params)
    nc = sim.info["nc"]
    # a block at level 2 or more whose particles are in the middle of their step
    key, lvl, ids = sim.debug("KEY"), sim.debug("BLK_LEVEL"), sim.debug("ID")
    level, _, _, val = decode_meta(sim.debug("META"))
    occ = np.unique(key)
    cand = [b for b in occ if lvl[b] >= 2 and np.count_nonzero((key == b) & (val > 1)) >= 4]
    assert cand, "the developed column should hold a slow block in mid-step"
    b = cand[len(cand) // 2]
    hit = ids[key == b]
    # 3 m/s along x: above level 2's Eq. 3 bound, below level 1's
    dv = np.zeros((sim.n, 3), np.float32)
    dv[hit, 0] = 3.0
    sim.add_velocity(dv)
    ref.v[:] = ref.v + dv.astype(np.float64)
    sim.advance(1)
    sim.sync()
    ref.step(1)
    snap = snapshot_after_step(sim)
    exp = check_structure(sim, cfg, snap)          # keys, order, levels, flags, lists bit-exact
    ring = np.intersect1d(ring_of(int(b), nc), np.unique(exp["keys"]))
    assert exp["lraw"][b] == 1 and np.all(exp["lvl"][ring] <= 1)
    level1, comp1, _, val1 = decode_meta(snap["META"])
    in_ring = np.isin(snap["KEY"], ring)
    pre = decode_meta(snap["PRE_META"])
    pre_val = pre[3][snap["PERM"]]
    pre_lvl = pre[0][snap["PERM"]]
    preempted = in_ring & (pre_val > 1) & (pre_lvl != level1)
    assert np.count_nonzero(preempted) >= 4
    # a pre-empted particle's next update: the next multiple of 2^level
    step = snap["STEP"]
    due = 2 ** level1[preempted] - step % 2 ** level1[preempted]
    assert np.all(comp1[preempted] == 1) and np.array_equal(val1[preempted], due)
    # the oracle's own run agrees on every particle's level and flag (caller order)
    gid = snap["ID"]
    assert np.array_equal(ref.level[gid], level1)
    assert np.array_equal(ref.compute[gid], comp1)
    sim.advance(4)
    st = sim.sync()
    ref.step(4)
    g = sim.state()
    dx = np.abs(g["pos"] - ref.x).max() / sc.params["spacing"]
    dvn = np.linalg.norm(g["vel"] - ref.v) / np.linalg.norm(ref.v)
    assert dx <= TRAJ_TOL and dvn <= TRAJ_TOL, (dx, dvn)
    assert st.active_total == sum(h["n_active"] for h in ref.history)
