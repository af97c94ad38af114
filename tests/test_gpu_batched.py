"""Batched scenes in one base step, and the launch-shape autotuner.

Independent dam breaks of uneven size are placed far apart in one particle
set, so that one graph replay advances all of them; each must evolve as it
does on its own.  The autotuner picks a launch shape without changing any
result.
"""
import numpy as np
import pytest

from paper_2009_14514_amd import _rts, scenes
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
    # 2 wave grids, 2 x 4 search shapes, 2 x 4 force shapes
    assert t["candidates"] == 18 and t["ms_per_step"] > 0
    assert tuned.tune()["grid_force"] == t["grid_force"]
    assert t["search_threads"] in (256, 512) and t["force_lanes"] in (4, 8)
    tuned.advance(30)
    tuned.sync()
    a, b = ref.state(), tuned.state()
    assert np.array_equal(a["pos"], b["pos"]) and np.array_equal(a["vel"], b["vel"])


SHAPES = [
    dict(search_threads=512, force_lanes=8, grid_search=768, grid_force=512),
    dict(search_threads=256, force_lanes=4, grid_search=1024, grid_force=768),
    dict(search_threads=512, force_lanes=4, grid_search=512, grid_force=256),
    dict(search_threads=256, force_lanes=8, grid_search=1536, grid_force=1024),
]


def test_launch_shapes_give_identical_bits():
    # workgroup size and count of the search, lanes per particle and
    # workgroup count of the force: the same 40 regional steps of a
    # 19,200-particle dam break bit for bit under each shape
    sc = scenes.dam_break_column(counts=(24, 40, 20), spacing=0.01, box=(0.6, 0.5, 0.3))
    runs = []
    for shape in SHAPES:
        sim = Simulation(sc)
        sim.set_tune(**shape)
        got = sim.tune()
        assert all(got[k] == v for k, v in shape.items()), (shape, got)
        sim.advance(40)
        st = sim.sync()
        runs.append((st, sim.state()))
        sim.close()
    st0, s0 = runs[0]
    assert st0.active_total > 0
    for (st, s), shape in zip(runs[1:], SHAPES[1:]):
        assert (st.active_total, st.inter_total) == (st0.active_total, st0.inter_total), shape
        for k in ("pos", "vel", "acc", "rho", "p", "level"):
            assert np.array_equal(s[k], s0[k]), (shape, k)


def test_launch_shape_out_of_range_is_refused():
    sim = Simulation(scenes.dam_break_small())
    for bad in (dict(search_threads=384), dict(force_lanes=16), dict(grid_force=0)):
        with pytest.raises(_rts.RtsError) as e:
            sim.set_tune(**bad)
        assert e.value.status == _rts.RTS_E_INVALID


def test_full_size_batch_structure_lists_and_sampled_density():
    """The 64-scene batch the benchmark times (2.78M particles), after the
    autotuner, as one particle set: keys, order, block starts, levels and
    flags bit-exact over every particle; lists of 1,000 sampled active
    particles bit-exact and inside their scene; their densities within 1e-5."""
    from parity import expected_structure, gpu_lists, oracle_density, oracle_lists, \
        snapshot_after_step
    import oracle
    sc = scenes.batched_dam_breaks()
    print(f"batch: {len(sc.parts)} scenes, {sc.n} particles", flush=True)
    sim = Simulation(sc)
    sim.autotune(steps=3)
    sim.advance(20)
    sim.sync()
    sim.advance(1)
    sim.sync()
    snap = snapshot_after_step(sim)
    cfg = oracle.cfg_from_params(sc.params)
    exp = expected_structure(cfg, snap)
    assert np.array_equal(snap["PERM"], exp["perm"])
    assert np.array_equal(snap["KEY"], exp["keys"])
    assert np.array_equal(snap["CELL_START"], exp["cell_start"])
    assert np.array_equal(snap["BLK_LEVEL"], exp["lvl"])
    from paper_2009_14514_amd.sim import decode_meta
    level, comp, _, _ = decode_meta(snap["META"])
    assert np.array_equal(comp, exp["compute"]) and np.array_equal(level, exp["level"])
    active = np.nonzero(comp)[0]
    rng = np.random.default_rng(3)
    sample = np.sort(rng.choice(active, size=min(1000, active.size), replace=False))
    want = np.zeros(sc.n, np.uint8)
    want[sample] = 1
    nbr, nnb = oracle_lists(cfg, snap, want)
    got, _ = gpu_lists(sim, snap, sample)
    owner = np.zeros(sc.n, np.int32)
    for k, (a, b) in enumerate(sc.parts):
        owner[a:b] = k
    ids = snap["ID"]
    for r, i in enumerate(sample):
        assert np.array_equal(got[r], nbr[i, :nnb[i]]), f"list of particle {i}"
        fl = got[r][got[r] < 0x80000000]
        assert np.all(owner[ids[fl]] == owner[ids[i]])
    rho_o, _ = oracle_density(cfg, snap, want)
    rel = np.abs(snap["POS"][sample, 3] - rho_o[sample]) / rho_o[sample]
    assert rel.max() <= 1e-5
    sim.close()


def test_device_generated_scenes_equal_the_host_generator():
    """rts_init_dam_break writes each scene's lattice column on the device:
    positions bit-exact against the seeded host generator, and the runs
    from both starts stay bitwise equal."""
    sc = small_batch()
    host = Simulation(sc)
    dev = Simulation(sc, device_init=True)
    a, b = host.state(), dev.state()
    assert np.array_equal(a["pos"], b["pos"]) and np.array_equal(a["vel"], b["vel"])
    host.advance(8)
    dev.advance(8)
    host.sync()
    dev.sync()
    a, b = host.state(), dev.state()
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    # a step ends the fresh state: the next column starts a new run of every scene
    c = sc.columns[0]
    dev.init_columns([c])
    with pytest.raises(Exception):
        dev.advance(1)              # the other scenes are not written yet
    dev.init_columns(sc.columns[1:])
    dev.advance(1)
    assert dev.sync().step == 1


def test_per_scene_counters_and_state_through_the_abi():
    sc = small_batch()
    sim = Simulation(sc)
    sim.advance(12)
    st = sim.sync()
    per = sim.scene_stats()
    assert len(per) == len(COUNTS)
    state = sim.state()
    for k, (a, b) in enumerate(sc.parts):
        assert per[k]["first"] == a and per[k]["n"] == b - a
        one = sim.scene_state(k)
        for f in ("pos", "vel", "rho", "p", "level"):
            assert np.array_equal(one[f], state[f][a:b]), (k, f)
        hist = np.bincount(state["level"][a:b], minlength=8)[:8]
        assert list(hist) == per[k]["level_hist"], k
        err = max(0.0, float(((state["rho"][a:b] - sc.params["rho0"]) / sc.params["rho0"]).max()))
        assert abs(per[k]["err_max_last"] - err) <= 1e-6
    assert sum(p["active_last"] for p in per) == st.active_last
    assert sum(p["inter_last"] for p in per) == st.inter_last
    assert [sum(p["level_hist"][l] for p in per) for l in range(8)] == list(st.level_hist)
    assert abs(max(p["err_max_last"] for p in per) - st.err_max_last) <= 1e-6
