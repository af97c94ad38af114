"""rts_create_static: a context in the library's static device workspace,
for callers that cannot allocate device memory.

Each call is checked against rts_create with a caller workspace on the same
scene: the same kernels run on the same inputs, so every output must agree
bit for bit.  The calls come in a row on the one array (a 19,200-particle
column, then a 4,096-particle column, then a 4,000-particle PCISPH scene),
each smaller than the last, so a context that relied on contents the
previous one left behind would differ.  Oversized scenes and a second live
context on the device are refused.
"""
import numpy as np
import pytest

from paper_2009_14514_amd import _rts, scenes
from paper_2009_14514_amd.sim import Simulation

pytestmark = pytest.mark.gpu


def run(sc, steps, static, **over):
    sim = Simulation(sc, static_workspace=static, **over)
    try:
        sim.advance(steps)
        st = sim.sync()
        s = sim.state()
        keys = sim.debug("KEY")
        return st, s, keys
    finally:
        sim.close()


CASES = [
    (lambda: scenes.dam_break_column(counts=(24, 40, 20), spacing=0.01, box=(0.6, 0.5, 0.3),
                                     c0=scenes.sound_speed_for_column(0.4, factor=10.0)), 40,
     dict(use_graph=0)),
    (scenes.dam_break_small, 25, dict(use_graph=1)),
    (scenes.pcisph_dam_break_small, 8, dict()),
]


def test_static_workspace_runs_equal_caller_workspace_runs():
    for make, steps, over in CASES:
        sc = make()
        st_a, a, ka = run(sc, steps, False, **over)
        st_b, b, kb = run(sc, steps, True, **over)
        assert (st_a.step, st_a.active_total, st_a.inter_total) == \
            (st_b.step, st_b.active_total, st_b.inter_total), sc.name
        assert st_b.status == 0
        for k in a:
            assert np.array_equal(a[k], b[k]), f"{sc.name}: {k}"
        assert np.array_equal(ka, kb), sc.name


def test_static_workspace_limits():
    big = scenes.dam_break_column()                 # 250,000 particles: 327 MiB of workspace
    with pytest.raises(_rts.RtsError) as e:
        Simulation(big, static_workspace=True)
    assert e.value.status == _rts.RTS_E_CAPACITY
    sc = scenes.dam_break_small()
    first = Simulation(sc, static_workspace=True)
    try:
        with pytest.raises(_rts.RtsError) as e:
            Simulation(sc, static_workspace=True)
        assert e.value.status == _rts.RTS_E_STATE
    finally:
        first.close()
    again = Simulation(sc, static_workspace=True)   # released by the close
    again.advance(2)
    assert again.sync().step == 2
    again.close()
