"""GPU edge cases of regional PCISPH.

An empty scene, a lone particle in free fall (with no neighbour the density
and pressure terms vanish and Algorithm 2's integration is symplectic Euler
under gravity: closed form and the oracle), ragged particle counts whose
neighbour lists must equal the oracle's bit for bit, and a neighbour-list
capacity overflow reported through the device status.
"""
import numpy as np
import pytest

import oracle
from paper_2009_14514_amd import _rts, scenes
from paper_2009_14514_amd.sim import Simulation, decode_meta, pcisph_lists

pytestmark = pytest.mark.gpu


def custom_scene(pos, vel=None):
    sc = scenes.pcisph_dam_break_small()
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    return scenes.Scene("custom", pos, np.zeros_like(pos) if vel is None else vel, sc.walls,
                        dict(sc.params))


def test_empty_scene_advances_time_only():
    sc = custom_scene(np.zeros((0, 3)))
    sim = Simulation(sc, n_fluid_max=16)
    sim.advance(4)
    st = sim.sync()
    assert st.pci_lists == 0
    assert st.time == pytest.approx(4 * sc.params["dt_base"], rel=1e-6)


def test_lone_particle_falls_freely():
    x0 = np.array([[0.4, 0.3, 0.15]])
    sc = custom_scene(x0)
    sim = Simulation(sc)
    steps = 12
    for _ in range(steps):
        sim.advance(1)
    st = sim.sync()
    s = sim.state()
    dt, g = sc.params["dt_base"], -9.81
    # v_k = k dt g, x_k = x_0 + dt^2 g k (k + 1) / 2
    assert s["vel"][0, 1] == pytest.approx(steps * dt * g, rel=1e-5)
    assert s["pos"][0, 1] == pytest.approx(x0[0, 1] + dt * dt * g * steps * (steps + 1) / 2,
                                           abs=1e-6)
    assert s["pos"][0, 0] == pytest.approx(x0[0, 0], abs=1e-7)
    ref = oracle.PCISPH(sc.params, sc.pos.astype(np.float32), vel=sc.vel,
                        walls=sc.walls.astype(np.float32))
    for _ in range(steps):
        ref.step()
    assert np.abs(s["pos"] - ref.in_caller_order(ref.x)).max() < 1e-6
    assert st.pci_errmax == 0.0


@pytest.mark.parametrize("n", [1, 2, 63, 65, 257, 1000])
def test_ragged_counts_lists_match_the_oracle(n):
    rng = np.random.default_rng(100 + n)
    # a cube holding n particles at about the rest spacing (0.02 m)
    side = max(0.05, (n * 0.02 ** 3) ** (1.0 / 3.0))
    pos = rng.uniform(0.05, 0.05 + side, size=(n, 3))
    sc = custom_scene(pos)
    over = dict(it_min=1, it_max=1)
    sim = Simulation(sc, **over)
    sim.assign_levels()
    before = {k: sim.debug(k) for k in ("POS", "META", "KEY", "CELL_START")}
    sim.advance(1)
    sim.sync()
    cfg = oracle.cfg_from_params(sc.params, **over)
    rows, counts = pcisph_lists(sim)
    level, comp, _, _ = decode_meta(before["META"])
    rings = np.where(level == 0, 2, 1).astype(np.uint8)
    st, nbr, nnb = oracle.pci_lists(cfg, before["POS"][:, :3], before["CELL_START"],
                                    before["KEY"], sim.debug("WALL_POS")[:, :3],
                                    sim.debug("WALL_CELL_START"), want=comp, rings=rings)
    assert st == 0
    assert np.array_equal(counts, nnb.astype(np.uint32))
    for i in range(n):
        assert np.array_equal(rows[i, :counts[i]], nbr[i, :nnb[i]]), f"list of particle {i}"


def test_list_capacity_overflow_is_reported():
    sc = scenes.pcisph_dam_break_small()
    sim = Simulation(sc, nbr_cap=9)            # about 45 neighbours at rest
    sim.advance(1)
    with pytest.raises(_rts.RtsError) as e:
        sim.sync()
    assert e.value.status == _rts.RTS_E_CAPACITY
    with pytest.raises(_rts.RtsError) as e:
        sim.advance(1)                          # state failed: refuse to go on
    assert e.value.status == _rts.RTS_E_STATE
    sim.set_state(sc.pos[:1] + 0.05, None)      # a fresh state clears the failure
    sim.advance(1)
    sim.sync()
