"""Full-size checks of regional PCISPH on the 1,000,188-particle double dam
break that the benchmark times, in the same launch configuration.

The major-step set-up (order, keys, block starts, regions before and after
dilation and R_min, observed blocks, flags) is compared bit for bit over
every particle and block; lists, the non-pressure acceleration, the
prediction and the density of the first correction iteration on 2,000
sampled particles, which the oracle computes one by one.
"""
import numpy as np
import pytest

import oracle
from paper_2009_14514_amd import scenes
from paper_2009_14514_amd.sim import Simulation, decode_meta, pcisph_lists

from test_gpu_pcisph import expected_major, region_validity

pytestmark = pytest.mark.gpu


def test_full_size_major_step_and_sampled_first_iteration():
    sc = scenes.double_dam_break()
    print(f"double dam break: {sc.n} particles, {sc.nw} wall particles", flush=True)
    over = dict(it_min=1, it_max=1)
    sim = Simulation(sc, **over)
    cfg = oracle.cfg_from_params(sc.params, **over)
    sim.assign_levels()
    exp = expected_major(cfg, sim)
    assert np.array_equal(sim.debug("PERM"), exp["perm"])
    assert np.array_equal(sim.debug("KEY"), exp["keys"])
    assert np.array_equal(sim.debug("CELL_START"), exp["start"])
    assert np.array_equal(sim.debug("BLK_LEVEL_RAW"), exp["raw"])
    assert np.array_equal(sim.debug("PCI_DILATED"), exp["dil"])
    assert np.array_equal(sim.debug("BLK_LEVEL"), exp["lvl"])
    occ = np.unique(exp["keys"])
    assert np.array_equal(sim.debug("PCI_OB")[occ], exp["ob"][occ])
    level, comp, _, val = decode_meta(sim.debug("META"))
    want_level = exp["lvl"][exp["keys"]].astype(np.int32)
    assert np.array_equal(level, want_level) and np.all(comp == 1)
    assert np.array_equal(val, region_validity(want_level, sim.sync().pci_major_len))

    before = {k: sim.debug(k) for k in ("POS", "VEL", "KEY", "CELL_START")}
    sim.advance(1)
    sim.sync()
    rng = np.random.default_rng(7)
    sample = np.sort(rng.choice(sc.n, size=2000, replace=False))
    want = np.zeros(sc.n, np.uint8)
    want[sample] = 1
    rings = np.where(level == 0, 2, 1).astype(np.uint8)
    wpos = sim.debug("WALL_POS")[:, :3]
    st, nbr, nnb = oracle.pci_lists(cfg, before["POS"][:, :3], before["CELL_START"],
                                    before["KEY"], wpos, sim.debug("WALL_CELL_START"),
                                    want=want, rings=rings)
    assert st == 0
    rows, counts = pcisph_lists(sim)
    assert np.array_equal(counts[sample], nnb[sample].astype(np.uint32))
    for i in sample:
        assert np.array_equal(rows[i, :counts[i]], nbr[i, :nnb[i]]), f"list of particle {i}"
    # non-pressure acceleration, prediction and density at the samples
    wx = wpos.astype(np.float64)
    x0 = before["POS"][:, :3].astype(np.float64)
    u0 = before["VEL"][:, :3].astype(np.float64)
    lists = np.zeros((sc.n, cfg.nbr_cap), np.uint32)
    lists[sample] = rows[sample]
    cnt = np.zeros(sc.n, np.int32)
    cnt[sample] = counts[sample]
    fvg = sim.debug("PCI_FVG")[:, :3].astype(np.float64)
    want_fvg = oracle.pci_nonpressure(cfg, x0, u0, wx, lists, cnt, which=want)
    g = np.asarray(cfg.g)
    assert np.abs(fvg[sample] - want_fvg[sample]).max() <= 1e-5 * np.abs(g).max()
    xs = sim.debug("PCI_XS")[:, :3].astype(np.float64)
    dt = oracle.derive(cfg).dt_base
    want_xs = x0[sample] + dt * (u0[sample] + dt * fvg[sample])
    assert np.abs(xs[sample] - want_xs).max() <= 1e-6 * np.abs(x0).max()
    rho = oracle.pci_density(cfg, xs, wx, lists, cnt, which=want)
    pv = sim.debug("PCI_PV").astype(np.float64)
    assert np.abs(pv[sample, 3] - rho[sample]).max() / cfg.rho0 <= 1e-5
    sim.close()
