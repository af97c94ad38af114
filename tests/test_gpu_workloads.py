"""Oracle parity of the paper's other WCSPH scenes and of the ablation.

* The double dam break and the dam break with a dropped block (the WCSPH
  rows of the paper's timing table), built by the same generators as the
  benchmark at sizes the oracle runs in seconds: 10 base steps of regional
  time stepping from a developed state (several levels present) within
  1e-4 spacings in position and 1e-4 in velocity (relative 2-norm), with
  the same active particles in every step.
* Regional time stepping without the Serna correction (Section 4.1, the
  correction's comparison figure): the same 10-step bound against the
  oracle run with the correction switched off.
"""
import numpy as np
import pytest

import oracle
from paper_2009_14514_amd import scenes
from paper_2009_14514_amd.sim import Simulation

from test_gpu_wcsph import TRAJ_TOL, f32, rts_scene

pytestmark = pytest.mark.gpu


def developed(sc, steps, **over):
    sim = Simulation(sc, **over)
    sim.advance(steps)
    sim.sync()
    s = sim.state()
    sim.close()
    return scenes.Scene(sc.name, s["pos"], s["vel"], sc.walls, sc.params)


def ten_steps(sc, **over):
    sim = Simulation(sc, **over)
    ref = oracle.WCSPH(sc.params, f32(sc.pos), vel=f32(sc.vel), walls=f32(sc.walls), **over)
    actives = []
    for _ in range(10):
        sim.advance(1)
        st = sim.sync()
        ref.step(1)
        actives.append((st.active_last, ref.history[-1]["n_active"]))
        assert list(st.level_hist)[:4] == ref.history[-1]["hist"][:4]
    g = sim.state()
    dx = np.abs(g["pos"] - ref.x).max() / sc.params["spacing"]
    dv = np.linalg.norm(g["vel"] - ref.v) / np.linalg.norm(ref.v)
    return dx, dv, actives, ref


def small_double_dam_break():
    # the benchmark generator at 2 x 12 x 24 x 12 = 6,912 particles
    return scenes.wcsph_double_dam_break(counts=(12, 24, 12), spacing=0.01, box=(0.6, 0.4, 0.3))


def small_block_drop():
    # the benchmark generator: a 14 x 20 x 14 column and an 8^3 block
    # released above the floor, 4,432 particles
    return scenes.block_drop(column=(14, 20, 14), block=(8, 8, 8), spacing=0.01,
                             box=(0.6, 0.5, 0.3), drop_at=(0.3, 0.3, 0.1))


@pytest.mark.parametrize("make", [small_double_dam_break, small_block_drop])
def test_second_workloads_follow_the_oracle(make):
    sc = developed(make(), 700)
    dx, dv, actives, ref = ten_steps(sc)
    assert all(a == b for a, b in actives), actives
    assert any(a < sc.n for a, _ in actives), "some particles should sit out a step"
    assert dx <= TRAJ_TOL and dv <= TRAJ_TOL, (dx, dv)


def test_without_serna_correction_follows_the_oracle():
    sc = developed(rts_scene(), 250, serna_correct=0)
    dx, dv, actives, ref = ten_steps(sc, serna_correct=0)
    assert all(a == b for a, b in actives), actives
    assert dx <= TRAJ_TOL and dv <= TRAJ_TOL, (dx, dv)
