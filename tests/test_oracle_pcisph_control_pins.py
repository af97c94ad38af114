"""Pins of the oracle's PCISPH control logic (no GPU).

Section "Regional Time Stepping with PCISPH", subsections "Extra Correction
Iterations", "Local Density Correction" and "Neighborhood Computation and
Updates", and Algorithms 2-3:

* the correction loop runs at least minIterations (3) iterations and until
  the maximum compression is below eta; after the three scheduled rows, an
  average compression of at least eta_T restarts the schedule (global
  iterations), otherwise local iterations correct S_e; local iterations that
  do not converge within a few (3) iterations switch back to global ones and
  the pressures return to their values from before the local phase; the
  switch back holds for the rest of the minor step (local correction is
  chosen once per minor step);
* a minor step with more than 6 global iterations ends its major step early;
  the following major steps are 2 minor steps long until 10 major steps in a
  row pass without such a minor step;
* region-1 particles rebuild their neighbourhood every minor step, region 2
  every second, regions 3 and 4 at the next major step;
* a particle that needs a smaller step takes its block and the neighbouring
  blocks to it.

Every expectation below is written out by hand from those statements (the
sequences of rows, counts and actions), not recomputed by the oracle's
formulas.  The global adaptive comparator's step, min(lambda_v r / c0,
lambda_f sqrt(r / max|a|)) (Eq. 1-2 applied to all particles), is pinned
against hand-computed values.
"""
import numpy as np
import pytest

import oracle as O
from paper_2009_14514_amd import scenes

KEEP, BACKUP, RESTORE = O.CTL_KEEP, O.CTL_BACKUP, O.CTL_RESTORE
R1, R2, R3, R4 = 0x1, 0x2, 0x4, 0x8
ALL = R1 | R2 | R3 | R4


def pcfg(**over):
    return O.cfg_from_params(scenes.pcisph_dam_break_small().params, **over)


def drive(cfg, errs, col=0, standard=False):
    """Runs the loop control over a list of (errmax, avg) pairs, one per
    iteration; returns the record of each iteration actually taken."""
    k = O.PciControl(cfg, standard)
    out = []
    err = np.inf
    for e, a in errs:
        if not k.more(err):
            break
        rec = dict(iter=k.iter, row=k.row, glob=k.k.global_, turn=k.turn(col))
        rec["action"] = k.after(e, a)
        out.append(rec)
        err = e
    return k, out, not k.more(err)


# --------------------------------------------------------------------------
# Algorithm 3: loop control
# --------------------------------------------------------------------------
def test_three_scheduled_rows_then_stop_when_converged():
    c = pcfg(eta=0.01, eta_T=0.0025)
    k, rec, stopped = drive(c, [(0.05, 0.001), (0.02, 0.001), (0.004, 0.001)] + [(0.5, 0.5)] * 5)
    assert stopped and len(rec) == 3
    assert [r["row"] for r in rec] == [1, 2, 3]
    assert all(r["glob"] == 1 and r["action"] == KEEP for r in rec)
    # column (a): two rows for every region, then region 1 (12/6/5/5 per major)
    assert [r["turn"] for r in rec] == [ALL, ALL, R1]
    assert (k.global_iters, k.resets, k.reverts, k.min_iter) == (3, 0, 0, 3)


@pytest.mark.parametrize("col,turns", [(0, [ALL, ALL, R1]), (1, [ALL, R1, R1]),
                                       (2, [ALL, R1 | R2, R1]), (3, [ALL, R1, R1])])
def test_rows_follow_the_column_of_the_minor_step(col, turns):
    c = pcfg()
    _, rec, _ = drive(c, [(0.0, 0.0)] * 3, col=col)
    assert [r["turn"] for r in rec] == turns


def test_at_least_min_iterations_even_when_converged_at_once():
    c = pcfg(eta=0.01, it_min=3)
    k, rec, stopped = drive(c, [(0.0, 0.0)] * 10)
    assert stopped and len(rec) == 3 and k.min_iter == 3


def test_global_error_restarts_the_schedule_after_every_extra_iteration():
    """Average >= eta_T: each iteration past the third sends the schedule back
    to its top row, so every extra iteration is row 1 (all regions)."""
    c = pcfg(eta=0.01, eta_T=0.0025, it_max=9)
    k, rec, stopped = drive(c, [(0.02, 0.003)] * 20)
    assert stopped and len(rec) == 9
    assert [r["row"] for r in rec] == [1, 2, 3, 1, 1, 1, 1, 1, 1]
    assert [r["turn"] for r in rec] == [ALL, ALL, R1] + [ALL] * 6
    assert all(r["glob"] == 1 and r["action"] == KEEP for r in rec)
    # a decision after each of iterations 3-9, the last one as well
    assert (k.global_iters, k.resets, k.reverts) == (9, 7, 0)
    assert k.min_iter == 3 + 7


def test_local_phase_reverts_after_local_fail_iterations():
    """Average < eta_T: local iterations on S_e (no region has the turn),
    a pressure snapshot when they begin, and after local_fail = 3 failed
    ones the pressures come back and the schedule restarts; no second local
    phase follows in the same minor step: every later extra iteration
    restarts the schedule (row 1, every region)."""
    c = pcfg(eta=0.01, eta_T=0.0025, it_max=12, local_fail=3)
    k, rec, stopped = drive(c, [(0.02, 0.001)] * 20)
    assert stopped and len(rec) == 12
    assert [r["glob"] for r in rec] == [1, 1, 1, 0, 0, 0, 1, 1, 1, 1, 1, 1]
    assert [r["row"] for r in rec] == [1, 2, 3, 4, 5, 6, 1, 1, 1, 1, 1, 1]
    assert [r["turn"] for r in rec] == [ALL, ALL, R1, 0, 0, 0, ALL, ALL, ALL, ALL, ALL, ALL]
    assert [r["action"] for r in rec] == [KEEP, KEEP, BACKUP, KEEP, KEEP, RESTORE,
                                          KEEP, KEEP, KEEP, KEEP, KEEP, KEEP]
    assert (k.global_iters, k.resets, k.reverts) == (9, 6, 1)


def test_a_new_minor_step_may_go_local_again():
    """The one-local-phase rule is per minor step: a fresh control (the next
    minor step) chooses local correction again."""
    c = pcfg(eta=0.01, eta_T=0.0025, it_max=8, local_fail=3)
    for _ in range(2):
        k, rec, _ = drive(c, [(0.02, 0.001)] * 20)
        assert [r["action"] for r in rec] == [KEEP, KEEP, BACKUP, KEEP, KEEP, RESTORE, KEEP, KEEP]


def test_a_local_phase_abandoned_for_the_mean_is_not_resumed():
    """The mean rising to eta_T ends the local phase too (revert and
    restart); when it falls back below eta_T the step stays global."""
    c = pcfg(eta=0.01, eta_T=0.0025, it_max=9)
    errs = [(0.02, 0.001)] * 4 + [(0.02, 0.003)] + [(0.02, 0.001)] * 10
    k, rec, stopped = drive(c, errs)
    assert stopped and len(rec) == 9
    assert [r["glob"] for r in rec] == [1, 1, 1, 0, 0, 1, 1, 1, 1]
    assert [r["action"] for r in rec] == [KEEP, KEEP, BACKUP, KEEP, RESTORE,
                                          KEEP, KEEP, KEEP, KEEP]
    assert (k.global_iters, k.resets, k.reverts) == (7, 5, 1)


@pytest.mark.parametrize("fail", [1, 2, 4])
def test_local_fail_sets_the_length_of_a_local_phase(fail):
    c = pcfg(eta=0.01, eta_T=0.0025, it_max=3 + fail + 1, local_fail=fail)
    k, rec, _ = drive(c, [(0.02, 0.001)] * 20)
    assert [r["glob"] for r in rec] == [1, 1, 1] + [0] * fail + [1]
    assert rec[2]["action"] == BACKUP and rec[2 + fail]["action"] == RESTORE
    assert k.reverts == 1


def test_local_phase_that_converges_keeps_its_pressures():
    c = pcfg(eta=0.01, eta_T=0.0025)
    k, rec, stopped = drive(c, [(0.02, 0.001)] * 4 + [(0.009, 0.001)] + [(0.5, 0.5)] * 5)
    assert stopped and len(rec) == 5
    assert [r["glob"] for r in rec] == [1, 1, 1, 0, 0]
    assert [r["action"] for r in rec] == [KEEP, KEEP, BACKUP, KEEP, KEEP]
    assert (k.global_iters, k.resets, k.reverts) == (3, 0, 0)


def test_global_error_during_a_local_phase_reverts_and_restarts():
    """The average rising to eta_T while local iterations run abandons them:
    pressures restored (a revert) and the schedule restarted (a reset)."""
    c = pcfg(eta=0.01, eta_T=0.0025)
    errs = [(0.02, 0.001)] * 4 + [(0.02, 0.003)] + [(0.001, 0.0)] * 5
    k, rec, stopped = drive(c, errs)
    assert [r["glob"] for r in rec] == [1, 1, 1, 0, 0, 1]
    assert [r["row"] for r in rec][-1] == 1
    assert [r["action"] for r in rec] == [KEEP, KEEP, BACKUP, KEEP, RESTORE, KEEP]
    assert (k.resets, k.reverts) == (1, 1)
    assert stopped and len(rec) == 6


def test_min_iterations_grow_with_each_extra_iteration():
    c = pcfg(eta=0.01, eta_T=0.0025)
    k, rec, stopped = drive(c, [(0.02, 0.001)] * 3 + [(0.001, 0.0)] + [(0.5, 0.5)] * 3)
    assert stopped and len(rec) == 4 and k.min_iter == 4


def test_iteration_cap():
    c = pcfg(eta=0.01, it_max=7)
    _, rec, stopped = drive(c, [(0.5, 0.5)] * 50)
    assert stopped and len(rec) == 7


def test_standard_pcisph_takes_every_particle_and_never_goes_local():
    c = pcfg(eta=0.01, eta_T=0.0025, it_max=8)
    k, rec, _ = drive(c, [(0.02, 0.001)] * 20, standard=True)
    assert len(rec) == 8
    assert all(r["turn"] == ALL and r["glob"] == 1 and r["action"] == KEEP for r in rec)
    assert (k.resets, k.reverts, k.global_iters) == (0, 0, 8)


# --------------------------------------------------------------------------
# major-step length (early end, 2-minor-step majors, return)
# --------------------------------------------------------------------------
def major_run(c, global_iters_per_minor, standard=False):
    s = O.OrcPciState()
    s.major_len = c.n_minor
    out = []
    for g in global_iters_per_minor:
        ends = O.pci_major_length(c, s, g, standard)
        out.append((ends, s.last_early_end, s.major_len, s.minor_in_major))
        if ends:
            s.major_excess = 0       # a new major step starts (Algorithm 2)
    return out


def test_overrun_in_the_second_minor_step_ends_the_major_step():
    c = pcfg(n_minor=4, global_limit=6, short_majors=10)
    out = major_run(c, [3, 7])
    assert out[0] == (0, 0, 4, 1)
    assert out[1] == (1, 1, 2, 0)          # early end; following majors 2 long


def test_short_majors_return_to_full_length_after_exactly_ten_clean_ones():
    c = pcfg(n_minor=4, global_limit=6, short_majors=10)
    out = major_run(c, [3, 7] + [3] * 2 * 10 + [3] * 4)
    after = out[2:]
    ends = [i for i, o in enumerate(after) if o[0]]
    # ten clean 2-step majors, then back to 4 minor steps
    assert ends[:10] == [1, 3, 5, 7, 9, 11, 13, 15, 17, 19]
    assert [after[e][2] for e in ends[:9]] == [2] * 9
    assert after[19][2] == 4
    assert after[23] == (1, 0, 4, 0)
    assert not any(o[1] for o in after)


def test_overrun_in_the_last_minor_step_is_no_early_end_but_shortens():
    c = pcfg(n_minor=4, global_limit=6, short_majors=10)
    out = major_run(c, [3, 3, 3, 7])
    assert out[3] == (1, 0, 2, 0)


def test_overrun_in_a_short_major_restarts_the_clean_count():
    c = pcfg(n_minor=4, global_limit=6, short_majors=3)
    out = major_run(c, [9] + [3] * 4 + [3, 8] + [3] * 6 + [3] * 4)
    lens = [o[2] for o in out]
    assert out[0] == (1, 1, 2, 0)
    assert lens[4] == 2                      # two clean short majors only
    assert out[6] == (1, 0, 2, 0)            # overrun at its last minor step
    assert lens[11] == 2 and lens[12] == 4   # three clean majors after it


def test_global_limit_is_a_strict_bound():
    c = pcfg(n_minor=4, global_limit=6)
    assert major_run(c, [6])[0] == (0, 0, 4, 1)
    assert major_run(c, [7])[0] == (1, 1, 2, 0)


def test_standard_pcisph_has_no_major_length_control():
    c = pcfg(n_minor=4, global_limit=6)
    s = O.OrcPciState()
    s.major_len = 1
    for g in (3, 20, 3):
        assert O.pci_major_length(c, s, g, True) == 1
        assert s.major_len == 1 and s.last_early_end == 0


# --------------------------------------------------------------------------
# neighbourhood cadence and smaller-step marking
# --------------------------------------------------------------------------
def test_region_validity_values():
    assert [O.pci_region_validity(r, 4) for r in (1, 2, 3, 4)] == [1, 2, 4, 4]
    assert [O.pci_region_validity(r, 2) for r in (1, 2, 3, 4)] == [1, 2, 2, 2]


def test_region_speed_bounds_at_the_scene_parameters():
    """Eq. 3 with alpha = 1, r = 2 s = 0.04 m, dt_b = 1e-3 s and beta_2..4 =
    0.4, 0.08, 0.016: region n holds speeds up to beta_n r / (n dt_b) =
    8, 1.0667 and 0.16 m/s; Eq. 2 with lambda_f = 0.25 bounds accelerations
    by lambda_f^2 r / (n dt_b)^2 = 625, 277.8 and 156.25 m/s^2."""
    info = O.derive(pcfg())
    assert np.sqrt(info.TV[1]) == pytest.approx(8.0, rel=1e-6)
    assert np.sqrt(info.TV[2]) == pytest.approx(0.04 * 0.08 / 3e-3, rel=1e-6)
    assert np.sqrt(info.TV[3]) == pytest.approx(0.16, rel=1e-6)
    assert np.sqrt(info.TA[1]) == pytest.approx(625.0, rel=1e-6)
    assert np.sqrt(info.TA[2]) == pytest.approx(0.0025 / 9e-6, rel=1e-6)
    assert np.sqrt(info.TA[3]) == pytest.approx(156.25, rel=1e-6)


def cube_of_blocks(c, lo, n):
    """One particle at the centre of each block of an n^3 cube of blocks whose
    lowest block has coordinates lo; returns (positions, block coordinates)."""
    info = O.derive(c)
    e = c.block_edge
    o = np.asarray(info.o, np.float64)
    coords = np.array([(lo[0] + i, lo[1] + j, lo[2] + k) for k in range(n) for j in range(n)
                       for i in range(n)], np.int64)
    pos = o[None, :] + (coords + 0.5) * e
    return pos, coords


def test_a_particle_needing_a_smaller_step_takes_its_block_and_neighbours():
    c = pcfg()
    info = O.derive(c)
    pos, coords = cube_of_blocks(c, (3, 3, 2), 5)
    n = pos.shape[0]
    key = O.keys(c, pos.astype(np.float32))
    nx, ny = info.nc[0], info.nc[1]
    assert np.array_equal(key, coords[:, 0] + nx * (coords[:, 1] + ny * coords[:, 2]))
    lvl = np.full(info.nblocks, O.EMPTY_BLOCK, np.uint8)
    lvl[key] = 3                                       # every block region 4
    ob = np.zeros(info.nblocks, np.uint8)
    region = np.full(n, 4, np.int32)
    validity = np.full(n, 3, np.int32)
    compute = np.zeros(n, np.uint8)
    vel = np.zeros((n, 3), np.float32)
    acc = np.zeros((n, 3), np.float32)
    acc[:, 1] = -9.81
    centre = int(np.where((coords == (6, 6, 5)).all(axis=1))[0][0])
    corner = int(np.where((coords == (3, 3, 2)).all(axis=1))[0][0])
    far = int(np.where((coords == (7, 3, 6)).all(axis=1))[0][0])
    vel[centre] = (12.0, 0.0, 0.0)                     # needs region 1
    vel[corner] = (0.0, 0.5, 0.0)                      # needs region 3
    vel[far] = (0.0, 0.1, 0.0)                         # region 4 suffices
    changed = O.pci_smaller_steps(c, key, vel, acc, 4, region, validity, compute, lvl, ob)
    assert changed == 1
    cheb_c = np.abs(coords - (6, 6, 5)).max(axis=1)
    cheb_k = np.abs(coords - (3, 3, 2)).max(axis=1)
    want_region = np.full(n, 4)
    want_region[cheb_k <= 1] = 3
    want_region[cheb_c <= 1] = 1
    assert np.array_equal(region, want_region)
    assert (cheb_c <= 1).sum() == 27 and (cheb_k <= 1).sum() == 8
    moved = want_region < 4
    assert np.array_equal(compute, moved.astype(np.uint8))
    assert np.array_equal(validity[cheb_c <= 1], np.ones(27))
    assert np.array_equal(validity[(cheb_k <= 1)], np.full(8, 4))   # region 3: the major step
    assert np.array_equal(validity[~moved], np.full((~moved).sum(), 3))
    assert np.array_equal(lvl[key], (want_region - 1).astype(np.uint8))
    # observed blocks: occupied, with an occupied neighbour of a smaller level
    for b in range(n):
        near = np.abs(coords - coords[b]).max(axis=1) <= 1
        assert ob[key[b]] == int((want_region[near] < want_region[b]).any()), coords[b]


def test_acceleration_alone_can_require_a_smaller_step():
    c = pcfg()
    info = O.derive(c)
    pos, coords = cube_of_blocks(c, (3, 3, 2), 3)
    n = pos.shape[0]
    key = O.keys(c, pos.astype(np.float32))
    lvl = np.full(info.nblocks, O.EMPTY_BLOCK, np.uint8)
    lvl[key] = 3
    ob = np.zeros(info.nblocks, np.uint8)
    region = np.full(n, 4, np.int32)
    validity = np.full(n, 4, np.int32)
    compute = np.zeros(n, np.uint8)
    vel = np.zeros((n, 3), np.float32)
    acc = np.zeros((n, 3), np.float32)
    acc[13] = (0.0, 400.0, 0.0)           # above 277.8 (region 3), below 625 (region 2)
    assert O.pci_smaller_steps(c, key, vel, acc, 4, region, validity, compute, lvl, ob) == 1
    assert np.all(region == 2) and np.all(compute == 1) and np.all(validity == 2)


def test_smaller_step_marking_never_raises_a_region():
    c = pcfg()
    info = O.derive(c)
    pos, coords = cube_of_blocks(c, (3, 3, 2), 3)
    n = pos.shape[0]
    key = O.keys(c, pos.astype(np.float32))
    lvl = np.full(info.nblocks, O.EMPTY_BLOCK, np.uint8)
    lvl[key] = 0
    ob = np.zeros(info.nblocks, np.uint8)
    region = np.ones(n, np.int32)
    validity = np.ones(n, np.int32)
    compute = np.zeros(n, np.uint8)
    vel = np.zeros((n, 3), np.float32)
    acc = np.zeros((n, 3), np.float32)
    assert O.pci_smaller_steps(c, key, vel, acc, 4, region, validity, compute, lvl, ob) == 0
    assert np.all(region == 1) and np.all(compute == 0) and np.all(lvl[key] == 0)


def test_particles_refresh_lists_at_their_region_cadence():
    """Four columns in regions 1-4 (none reaches another or a wall in the
    steps checked): in the second major step, a particle rebuilds its list in
    minor step j = 0 always, and in j = 1, 2, 3 only if it is in region 1,
    or in region 2 at j = 2."""
    sc = scenes.pcisph_thrown_columns(wall_gap=3.0)
    sim = O.PCISPH(sc.params, sc.pos, vel=sc.vel, walls=sc.walls)
    sim.step(4)
    assert sim.state.minor_in_major == 0
    regions = None
    for j in range(4):
        if j == 1:
            regions = sim.region.copy()
        comp = sim.compute.copy()
        sim.step()
        h = sim.history[-1]
        assert h["lists"] == int(comp.sum())
        if j == 0:
            assert np.all(comp == 1)
            continue
        reg = sim.region
        assert sorted(np.bincount(reg, minlength=5)[1:]) == [216] * 4
        want = (reg == 1) | ((reg == 2) & (j == 2))
        assert np.array_equal(comp.astype(bool), want), f"minor step {j}"
    assert np.array_equal(regions, sim.region)      # no smaller step was forced
    assert sim.history[-1]["lists"] == 216           # region 1 alone at j = 3


# --------------------------------------------------------------------------
# whole minor steps with forced control paths (trace of every iteration)
# --------------------------------------------------------------------------
def traced(steps, **over):
    sc = scenes.pcisph_thrown_columns(wall_gap=3.0)
    sim = O.PCISPH(sc.params, sc.pos, vel=sc.vel, walls=sc.walls, **over)
    sim.enable_trace(pressures=True)
    sim.step(steps)
    return sim


def test_forced_local_phases_restore_the_pressures_bit_for_bit():
    """eta tiny (never converged) with eta_T above any average: every minor
    step runs it_max = 12 iterations as 3 scheduled rows, 3 local, a revert,
    then 6 global restarts (row 1, every particle)."""
    sim = traced(2, eta=1e-9, eta_T=1.0, it_max=12)
    for h in sim.history:
        tr = h["trace"]
        assert [t["glob"] for t in tr] == [1, 1, 1, 0, 0, 0, 1, 1, 1, 1, 1, 1]
        assert [t["action"] for t in tr] == [KEEP, KEEP, BACKUP, KEEP, KEEP, RESTORE,
                                             KEEP, KEEP, KEEP, KEEP, KEEP, KEEP]
        assert [t["row"] for t in tr][6:] == [1] * 6
        assert all(t["n_density"] == sim.state.n for t in tr[6:])
        assert (h["iters"], h["global_iters"], h["resets"], h["reverts"]) == (12, 9, 6, 1)
        P = h["trace_p"]
        # the snapshot is the pressure after iteration 3; the revert after
        # iteration 6 brings it back exactly, though iterations 4-6 moved it
        assert np.array_equal(P[5], P[2])
        assert not np.array_equal(P[3], P[2])
        assert not np.array_equal(P[6], P[5])
        # local iterations: no region has the turn; the pressure force is
        # evaluated on S_e alone, the density on S_e and the observed blocks
        for t in tr:
            if t["glob"] == 0:
                assert t["turn"] == 0 and t["n_force"] == t["n_se"]
                assert t["n_density"] >= t["n_se"]


def test_forced_global_restarts_every_extra_iteration():
    sim = traced(2, eta=1e-9, eta_T=0.0, it_max=8)
    for h in sim.history:
        tr = h["trace"]
        assert [t["row"] for t in tr] == [1, 2, 3, 1, 1, 1, 1, 1]
        assert all(t["glob"] == 1 and t["action"] == KEEP for t in tr)
        assert all(t["n_density"] == sim.state.n for t in tr[3:])   # every region
        assert (h["iters"], h["global_iters"], h["resets"], h["reverts"]) == (8, 8, 6, 0)


def test_forced_overrun_ends_every_major_step_after_one_minor_step():
    """More than global_limit global iterations in every minor step: each
    ends its major step, so every minor step starts a major step (grid,
    regions, every list rebuilt) and the length stays 2."""
    sim = traced(4, eta=1e-9, eta_T=0.0, it_max=8, global_limit=6)
    for h in sim.history:
        assert h["early_end"] == 1 and h["major_len"] == 2 and h["minor_in_major"] == 0
        assert h["lists"] == sim.state.n


def test_return_to_long_major_steps_after_clean_ones_end_to_end():
    """Two overrun minor steps, then a tolerance every step meets: the
    following majors are 2 minor steps long until short_majors = 2 clean
    ones have passed, then 4 again."""
    sc = scenes.pcisph_thrown_columns(wall_gap=3.0)
    sim = O.PCISPH(sc.params, sc.pos, vel=sc.vel, walls=sc.walls, eta=1e-9, eta_T=0.0,
                   it_max=8, short_majors=2)
    sim.step(1)
    assert sim.history[-1]["early_end"] == 1 and sim.state.major_len == 2
    sim.cfg.eta = 1.0                      # from now on every minor step converges
    sim.step(8)
    lens = [h["major_len"] for h in sim.history[1:]]
    ends = [h["minor_in_major"] == 0 for h in sim.history[1:]]
    assert ends[:4] == [False, True, False, True]
    assert lens[:4] == [2, 2, 2, 4]
    assert lens[4:] == [4, 4, 4, 4] and ends[4:] == [False, False, False, True]
    assert all(h["early_end"] == 0 and h["iters"] == 3 for h in sim.history[1:])


# --------------------------------------------------------------------------
# global adaptive WCSPH comparator
# --------------------------------------------------------------------------
def test_global_adaptive_step_hand_values():
    """r = r_crit = 2 s = 0.02 m (250k dam break), c0 = 88.58893836 m/s,
    lambda_v = 0.4, lambda_f = 0.25: the sound-speed bound is
    0.4 * 0.02 / 88.58893836 = 9.0304728199e-5 s; an acceleration of
    |a| = 2000 m/s^2 gives 0.25 sqrt(0.02 / 2000) = 7.90569415e-4 s (the
    sound bound wins) and |a| = 5e5 m/s^2 gives 0.25 sqrt(4e-8) = 5e-5 s."""
    p = scenes.dam_break_column(c0=88.58893836, mode="global_adaptive").params
    c = O.cfg_from_params(p)
    assert c.r_crit == pytest.approx(0.02)
    a = np.zeros((5, 3))
    assert O.adaptive_dt(c, a) == pytest.approx(9.0304728199e-5, rel=1e-9)
    a[2] = (0.0, -2000.0, 0.0)
    assert O.adaptive_dt(c, a) == pytest.approx(9.0304728199e-5, rel=1e-9)
    a[3] = (3e5, 4e5, 0.0)                 # |a| = 5e5
    assert O.adaptive_dt(c, a) == pytest.approx(5e-5, rel=1e-12)
    # Eq. 2 alone (a sound speed too low to bind)
    c.c0 = 1.0
    a[3] = (0.0, 2000.0, 0.0)
    assert O.adaptive_dt(c, a) == pytest.approx(7.90569415e-4, rel=1e-8)


def test_global_adaptive_run_takes_the_rule_each_step():
    """The oracle's global adaptive run advances by exactly that step."""
    sc = scenes.dam_break_column(counts=(10, 16, 8), mode="global_adaptive")
    sim = O.WCSPH(sc.params, sc.pos, walls=sc.walls)
    for _ in range(4):
        t0 = sim.t
        sim.step()
        # the step is taken after the corrector with the new accelerations
        assert sim.t - t0 == pytest.approx(O.adaptive_dt(sim.cfg, sim.a), rel=1e-12)
