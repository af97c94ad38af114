"""Pins of the oracle's adaptive base step for regional PCISPH (no GPU).

The paper's conclusions suggest adjusting the PCISPH base step between major
steps in the manner of global adaptive PCISPH.  The reading built here: the
correction effort of a major step steers the next one's base step, capped by
Eq. 3 (with beta_2) and Eq. 2 for the fastest particle, and a correction
that fails to converge rolls its major step back and restarts it with a
shorter step.  The pins: the step limits as the displacement and
acceleration bounds they stand for, the growth sequence on a calm start,
equivalence with the fixed-step run where the rule must not act, and a
roll-back that lands exactly on the fixed-step run at the shortened step.
"""
import numpy as np
import pytest

import oracle as O
from paper_2009_14514_amd import scenes


def run(sc, steps, **over):
    sim = O.PCISPH(sc.params, sc.pos, vel=sc.vel, walls=sc.walls, **over)
    sim.step(steps)
    return sim


def f32_norm2_max(a):
    a = np.asarray(a, np.float64).astype(np.float32)
    return float(np.max((a[:, 0] * a[:, 0] + a[:, 1] * a[:, 1]) + a[:, 2] * a[:, 2]))


def accepted(sim):
    return [h for h in sim.history if not h["rollback"]]


@pytest.mark.parametrize("seed", range(4))
def test_next_step_respects_the_displacement_and_acceleration_bounds(seed):
    """Whatever the effort, the next base step lets the fastest particle
    cross at most alpha beta_2 r (Eq. 3) and keeps dt^2 |a|max within
    lambda_f^2 r (Eq. 2), unless the floor dt_min is what holds it up; it
    never leaves [dt_min, dt_max]."""
    rng = np.random.default_rng(seed)
    c = O.cfg_from_params(scenes.pcisph_dam_break_small().params, pci_adapt_dt=1)
    r, lo, hi = c.r_crit, 0.25 * c.dt_base, 4.0 * c.dt_base
    for _ in range(200):
        dt = float(rng.uniform(lo, hi))
        v2 = np.float32(10.0 ** rng.uniform(-3, 3))
        a2 = np.float32(10.0 ** rng.uniform(0, 9))
        nxt = O.pci_next_dt(c, dt, int(rng.integers(3, 12)), int(rng.integers(0, 2)), v2, a2)
        assert lo <= nxt <= hi
        if nxt > lo:
            assert nxt * np.sqrt(np.float64(v2)) <= c.alpha_rts * c.beta2 * r * (1 + 1e-12)
            assert nxt * nxt * np.sqrt(np.float64(a2)) <= c.lambda_f ** 2 * r * (1 + 1e-12)


def test_effort_steers_the_step():
    """By default a major step whose minor steps all converged in it_min
    iterations grows the step, one needing more (or overrunning the global
    limit) shrinks it; with a band between the two thresholds the step holds
    (with no speed or acceleration to cap it)."""
    c = O.cfg_from_params(scenes.pcisph_dam_break_small().params, pci_adapt_dt=1)
    dt = c.dt_base
    assert O.pci_next_dt(c, dt, 3, 1, 0.0, 0.0) == pytest.approx(0.95 * dt, rel=1e-15)
    assert O.pci_next_dt(c, dt, 4, 0, 0.0, 0.0) == pytest.approx(0.95 * dt, rel=1e-15)
    assert O.pci_next_dt(c, dt, 3, 0, 0.0, 0.0) == pytest.approx(1.02 * dt, rel=1e-15)
    band = O.cfg_from_params(scenes.pcisph_dam_break_small().params, pci_adapt_dt=1,
                             pci_shrink_iters=5)
    assert O.pci_next_dt(band, dt, 4, 0, 0.0, 0.0) == dt
    assert O.pci_next_dt(band, dt, 5, 0, 0.0, 0.0) == dt
    assert O.pci_next_dt(band, dt, 6, 0, 0.0, 0.0) == pytest.approx(0.95 * dt, rel=1e-15)
    assert O.pci_next_dt(c, 0.26 * dt, 9, 1, 0.0, 0.0) == 0.25 * dt     # floor
    assert O.pci_next_dt(c, 3.95 * dt, 3, 0, 0.0, 0.0) == 4.0 * dt      # ceiling
    assert O.pci_next_dt(c, dt, 3, 0, 0.0, 0.0) == O.pci_next_dt(c, dt, 2, 0, 0.0, 0.0)


def test_calm_start_grows_geometrically_at_major_boundaries():
    """The first 40 ms of the small double dam break converge in the minimum
    three iterations, so major step k runs at dt0 1.02^k, the same for all
    its minor steps, and simulated time is the sum of the steps."""
    sc = scenes.pcisph_dam_break_small(dt_base=1e-3)
    sim = run(sc, 24, pci_adapt_dt=1)
    hs = accepted(sim)
    assert len(hs) == 24 and all(h["iters"] == 3 for h in hs)
    for k, h in enumerate(hs):
        assert h["dt"] == pytest.approx(1e-3 * 1.02 ** (k // 4), rel=1e-12), k
    assert sim.t == pytest.approx(sum(h["dt"] for h in hs), rel=1e-12)
    # the maxima the rule read at the last major end, recomputed from the state
    assert hs[-1]["minor_in_major"] == 0
    assert hs[-1]["v2max"] == f32_norm2_max(sim.v)
    assert hs[-1]["a2max"] == f32_norm2_max(sim.fvg + sim.fp)


def test_eq3_caps_a_fast_scene():
    """Columns thrown at 20 m/s: after the first major step the base step is
    the Eq. 3 limit, so the fastest particle crosses exactly alpha beta_2 r
    per base step."""
    sc = scenes.pcisph_dam_break_small(dt_base=1e-3, v0=20.0)
    sim = run(sc, 4, pci_adapt_dt=1)
    h = sim.history[-1]
    assert h["minor_in_major"] == 0
    vmax = np.sqrt(np.float64(f32_norm2_max(sim.v)))
    c = sim.cfg
    assert h["dt_next"] < 1e-3
    assert h["dt_next"] * vmax == pytest.approx(c.alpha_rts * c.beta2 * c.r_crit, rel=1e-12)


def test_rule_that_cannot_act_leaves_the_fixed_step_run_unchanged():
    """Factors of one and caps that do not bind: the adaptive run, snapshots
    and all, is the fixed-step run bit for bit."""
    sc = scenes.pcisph_dam_break_small(dt_base=1e-3)
    a = run(sc, 24, pci_adapt_dt=1, pci_grow=1.0, pci_shrink=1.0)
    b = run(sc, 24)
    assert np.array_equal(a.in_caller_order(a.x), b.in_caller_order(b.x))
    assert np.array_equal(a.in_caller_order(a.v), b.in_caller_order(b.v))
    assert [h["iters"] for h in a.history] == [h["iters"] for h in b.history]


def test_rollback_lands_on_the_fixed_run_at_the_shortened_step():
    """A tolerance no correction reaches within four iterations: the first
    major step is rolled back at dt0 and at dt0/2 (each roll-back halves the
    step), then accepted at the floor
    dt0/4; the run is then the fixed-step run at dt0/4 bit for bit, so the
    roll-back restored every particle array and counter it needs."""
    sc = scenes.pcisph_dam_break_small(dt_base=1e-3)
    strict = dict(eta=1e-7, it_max=4)
    a = run(sc, 8, pci_adapt_dt=1, pci_grow=1.0, pci_dt_min=2.5e-4, **strict)
    assert [h["rollback"] for h in a.history[:3]] == [1, 1, 0]
    assert a.state.rollbacks == 2
    b = run(scenes.pcisph_dam_break_small(dt_base=2.5e-4), 8, **strict)
    assert a.t == pytest.approx(8 * 2.5e-4, rel=1e-12)
    assert np.array_equal(a.in_caller_order(a.x), b.in_caller_order(b.x))
    assert np.array_equal(a.in_caller_order(a.v), b.in_caller_order(b.v))
    assert [h["iters"] for h in accepted(a)] == [h["iters"] for h in b.history]
