"""GPU parity of the adaptive base step of regional PCISPH against the oracle.

The same seeded small double dam break runs on both sides: the base step of
every accepted minor step, the iteration counts, the roll-backs and the
final positions must agree.
"""
import numpy as np
import pytest

import oracle
from paper_2009_14514_amd import scenes
from paper_2009_14514_amd.sim import Simulation

pytestmark = pytest.mark.gpu


def both(sc, **over):
    sim = Simulation(sc, **over)
    ref = oracle.PCISPH(sc.params, sc.pos.astype(np.float32), vel=sc.vel,
                        walls=sc.walls.astype(np.float32), **over)
    return sim, ref


@pytest.mark.parametrize("v0,steps", [(0.0, 24), (20.0, 8)])
def test_adaptive_steps_follow_the_oracle(v0, steps):
    """Calm start (the step grows at every major boundary) and columns thrown
    at each other at 20 m/s (Eq. 3 caps the step from the second major step
    on; eight steps end before they meet)."""
    sc = scenes.pcisph_dam_break_small(dt_base=1e-3, v0=v0)
    sim, ref = both(sc, pci_adapt_dt=1)
    for k in range(steps):
        sim.advance(1)
        st = sim.sync()
        ref.step()
        h = ref.history[-1]
        assert st.pci_iters == h["iters"], f"step {k}"
        assert st.dt_last == pytest.approx(h["dt"], rel=1e-5), f"step {k}"
        assert st.pci_dt_next == pytest.approx(h["dt_next"], rel=1e-5), f"step {k}"
        assert st.pci_major_len == h["major_len"] and st.pci_minor_in_major == h["minor_in_major"]
    assert st.time == pytest.approx(ref.t, rel=1e-5)
    if v0 > 0.0:
        assert st.dt_last < 1e-3        # the cap acted
    x_gpu = sim.state()["pos"]
    x_ref = ref.in_caller_order(ref.x)
    assert np.abs(x_gpu - x_ref).max() <= 1e-4 * sc.params["spacing"]
    sim.close()


def test_rollback_matches_the_oracle_and_the_fixed_step_run():
    """A tolerance no correction reaches in four iterations: two roll-backs on
    both sides, then the run at the floor dt0/4 equals the GPU's own
    fixed-step run at dt0/4 bit for bit.  (Positions are not compared with
    the oracle here: at a tolerance of 1e-7 membership of S_e, error above
    half of it, is decided by rounding.)"""
    strict = dict(eta=1e-7, it_max=4)
    sc = scenes.pcisph_dam_break_small(dt_base=1e-3)
    sim, ref = both(sc, pci_adapt_dt=1, pci_grow=1.0, pci_dt_min=2.5e-4, **strict)
    sim.advance(8)
    st = sim.sync()
    ref.step(8)
    assert st.pci_rollbacks == ref.state.rollbacks == 2
    assert st.step == 8
    assert st.time == pytest.approx(8 * 2.5e-4, rel=1e-12)
    x = sim.state()["pos"]
    fixed = Simulation(scenes.pcisph_dam_break_small(dt_base=2.5e-4), **strict)
    fixed.advance(8)
    fixed.sync()
    assert np.array_equal(x, fixed.state()["pos"])
    sim.close()
    fixed.close()
