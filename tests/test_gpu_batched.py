"""Batched scenes in one base step, and the launch-shape autotuner.

Independent dam breaks of uneven size are placed far apart in one particle
set, so that one graph replay advances all of them; each must evolve as it
does on its own.  The autotuner picks a launch shape without changing any
result.
"""
import numpy as np
import pytest

from paper_2009_14514_amd import scenes
from paper_2009_14514_amd.sim import Simulation, neighbour_lists

pytestmark = pytest.mark.gpu

COUNTS = [(10, 20, 10), (14, 8, 14), (6, 24, 6), (20, 10, 8)]


def small_batch():
    return scenes.batched_dam_breaks(n_scenes=4, counts=COUNTS, box=(0.6, 0.5, 0.3),
                                     spacing=0.02)


def test_batched_scenes_evolve_as_they_do_alone():
    sc = small_batch()
    steps = 12
    sim = Simulation(sc)
    sim.advance(steps)
    sim.sync()
    pos = sim.state()["pos"]
    s = sc.params["spacing"]
    for k, sub in enumerate(sc.subscenes):
        alone = Simulation(sub)
        alone.advance(steps)
        alone.sync()
        a, b = sc.parts[k]
        moved = pos[a:b] - np.asarray(sc.offsets[k], np.float32)[None, :]
        assert np.abs(moved - alone.state()["pos"]).max() <= 1e-4 * s, f"scene {k}"
        alone.close()


def test_batched_neighbour_lists_stay_inside_their_scene():
    sc = small_batch()
    sim = Simulation(sc)
    sim.advance(1)          # the first step evaluates every particle
    sim.sync()
    owner = np.zeros(sc.n, np.int32)
    for k, (a, b) in enumerate(sc.parts):
        owner[a:b] = k
    wall_owner = np.repeat(np.arange(len(COUNTS)), sc.nw // len(COUNTS))
    ids = sim.debug("ID")
    wids = sim.debug("WALL_ID")
    rows, counts = neighbour_lists(sim)
    checked = 0
    for i in np.nonzero(counts)[0]:
        lst = rows[i, :counts[i]]
        fl = lst[lst < 0x80000000]
        wl = lst[lst >= 0x80000000] & 0x7FFFFFFF
        me = owner[ids[i]]
        assert np.all(owner[ids[fl]] == me)
        assert np.all(wall_owner[wids[wl]] == me)
        checked += 1
    assert checked > 100


def test_autotune_keeps_results_bitwise():
    sc = scenes.dam_break_column(counts=(24, 40, 20), spacing=0.01, box=(0.6, 0.5, 0.3))
    ref = Simulation(sc)
    ref.advance(30)
    ref.sync()
    tuned = Simulation(sc)
    t = tuned.autotune(steps=3)
    assert t["candidates"] == 32 and t["ms_per_step"] > 0
    assert tuned.tune()["grid_force"] == t["grid_force"]
    tuned.advance(30)
    tuned.sync()
    a, b = ref.state(), tuned.state()
    assert np.array_equal(a["pos"], b["pos"]) and np.array_equal(a["vel"], b["vel"])
