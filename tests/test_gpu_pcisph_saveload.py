"""PCISPH save / load: a run saved in the middle of a major step and
restored into a fresh context continues bit for bit (Algorithms 2-3 keep
their state across minor steps: the major step's grid and regions, lists of
particles not due for a rebuild, non-pressure accelerations, the position
in the major step, the major-step length and the clean-major counter)."""
import numpy as np
import pytest

from paper_2009_14514_amd import scenes
from paper_2009_14514_amd.sim import Simulation

pytestmark = pytest.mark.gpu

FIELDS = ("step", "time", "pci_iters", "pci_global_iters", "pci_resets", "pci_reverts",
          "pci_lists", "pci_major_len", "pci_minor_in_major", "pci_iters_total",
          "pci_rollbacks", "pci_dt_next")


@pytest.mark.parametrize("make,over,first", [
    (scenes.pcisph_thrown_columns, dict(), 8),                  # 2-minor-step majors by then
    (scenes.pcisph_thrown_columns, dict(short_majors=2), 8),
    (scenes.pcisph_dam_break_small, dict(mode="global_fixed"), 9),
    (scenes.pcisph_dam_break_small, dict(pci_adapt_dt=1, dt_base=1e-3), 9),
])
def test_saved_run_continues_bitwise(make, over, first):
    sc = make()
    a = Simulation(sc, **over)
    a.advance(20)
    sa = a.sync()
    b = Simulation(sc, **over)
    b.advance(first)
    sb = b.sync()
    # saved inside a major step (standard PCISPH: every minor step is one)
    assert sb.pci_minor_in_major != 0 or over.get("mode") == "global_fixed"
    buf = b.save()
    b.close()
    c = Simulation(sc, **over)
    c.load(buf)
    c.advance(20 - first)
    sc_ = c.sync()
    for f in FIELDS:
        assert getattr(sa, f) == getattr(sc_, f), f
    assert list(sa.level_hist) == list(sc_.level_hist)
    xa, xc = a.state(), c.state()
    for k in xa:
        assert np.array_equal(xa[k], xc[k]), k


def test_load_refuses_a_state_of_another_configuration():
    from paper_2009_14514_amd import _rts
    sc = scenes.pcisph_dam_break_small()
    b = Simulation(sc)
    b.advance(3)
    buf = b.save()
    other = Simulation(sc, mode="global_fixed")
    with pytest.raises(_rts.RtsError) as e:
        other.load(buf)
    assert e.value.status == _rts.RTS_E_INVALID
