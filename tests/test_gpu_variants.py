"""Variants the paper describes, and its second WCSPH workloads.

* Without the Serna correction (the ablation of Section 4) the density error
  and the evaluated work grow.
* PCISPH with two-layer neighbour search for regions 1 and 2 (the paper's
  comparison figure) builds the same lists as the oracle.
* The double dam break and the block drop run their first steps within the
  compression bound under regional stepping.
"""
import numpy as np
import pytest

import oracle
from paper_2009_14514_amd import scenes
from paper_2009_14514_amd.sim import Simulation, decode_meta, pcisph_lists

pytestmark = pytest.mark.gpu


def test_without_serna_correction_errors_and_work_grow():
    sc = scenes.dam_break_column(counts=(24, 40, 20), spacing=0.01, box=(0.6, 0.5, 0.3))
    out = {}
    for corr in (1, 0):
        sim = Simulation(sc, serna_correct=corr)
        sim.advance(400)
        st = sim.sync()
        out[corr] = (st.err_max_run, st.active_total)
        sim.close()
    assert out[0][0] > 2.0 * out[1][0]
    assert out[0][1] > out[1][1]


def test_two_layer_search_for_regions_one_and_two():
    sc = scenes.pcisph_dam_break_small(v0=1.5)          # every block in region 2
    over = dict(it_min=1, it_max=1, two_ring_levels=2)
    sim = Simulation(sc, **over)
    sim.assign_levels()
    before = {k: sim.debug(k) for k in ("POS", "META", "KEY", "CELL_START")}
    sim.advance(1)
    sim.sync()
    rows, counts = pcisph_lists(sim)
    level, comp, _, _ = decode_meta(before["META"])
    assert np.all(level == 1)
    cfg = oracle.cfg_from_params(sc.params, **over)
    st, nbr, nnb = oracle.pci_lists(cfg, before["POS"][:, :3], before["CELL_START"], before["KEY"],
                                    sim.debug("WALL_POS")[:, :3], sim.debug("WALL_CELL_START"),
                                    want=comp, rings=np.full(sim.n, 2, np.uint8))
    assert st == 0 and np.array_equal(counts, nnb.astype(np.uint32))
    for i in range(sim.n):
        assert np.array_equal(rows[i, :counts[i]], nbr[i, :nnb[i]])


@pytest.mark.parametrize("make", [scenes.wcsph_double_dam_break, scenes.block_drop])
def test_second_workloads_stay_within_the_bound(make):
    sc = make()
    sim = Simulation(sc)
    sim.advance(200)
    st = sim.sync()
    assert st.err_max_run < 0.01
    assert 0 < st.active_total < 200 * sc.n
