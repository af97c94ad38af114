"""Pins of the CPU oracle against mathematics and the paper (no GPU).

Each test checks the oracle against something other than itself: closed
forms, quadrature, brute force, library routines, physical invariants, or
the constants the paper prints (tests/golden/paper_constants.json).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2009_14514_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def fused_d2(d):
    """Squared distance as the method's float predicate forms it:
    fma(dz, dz, fma(dy, dy, dx*dx)), each fused step rounded once (emulated
    through double, where the products of floats are exact)."""
    d = np.asarray(d, np.float32).astype(np.float64)
    xx = (d[:, 0] * d[:, 0]).astype(np.float32).astype(np.float64)
    s = (d[:, 1] * d[:, 1] + xx).astype(np.float32).astype(np.float64)
    return (d[:, 2] * d[:, 2] + s).astype(np.float32)


def params(**over):
    sc = scenes.dam_break_small()
    p = dict(sc.params)
    p.update(over)
    return p


def cfg(**over):
    return O.cfg_from_params(params(**over))


# --------------------------------------------------------------------------
# kernel
# --------------------------------------------------------------------------
def test_kernel_integrates_to_one():
    c = cfg()
    h = c.h
    r = np.linspace(0.0, 2.0 * h, 40001)
    f = np.array([4.0 * math.pi * x * x * O.kernel_W(c, x) for x in r])
    dr = r[1] - r[0]
    simpson = dr / 3.0 * (f[0] + f[-1] + 4.0 * f[1:-1:2].sum() + 2.0 * f[2:-1:2].sum())
    assert abs(simpson - 1.0) < 1e-10


def test_kernel_closed_form_and_continuity():
    c = cfg()
    h = c.h
    assert O.kernel_W(c, 0.0) == pytest.approx(1.0 / (math.pi * h ** 3), rel=1e-15)
    assert O.kernel_W(c, 2.0 * h) == 0.0
    assert O.kernel_W(c, 2.5 * h) == 0.0
    for q in (1.0, 2.0):
        lo, hi = O.kernel_W(c, (q - 1e-9) * h), O.kernel_W(c, (q + 1e-9) * h)
        assert abs(lo - hi) < 1e-6 * O.kernel_W(c, 0.0)
    assert O.kernel_dWdr(c, 0.0) == 0.0
    d1, d2 = O.kernel_dWdr(c, (1 - 1e-9) * h), O.kernel_dWdr(c, (1 + 1e-9) * h)
    assert abs(d1 - d2) < 1e-6 * abs(d1)


def test_kernel_derivative_matches_finite_difference():
    c = cfg()
    h = c.h
    for q in np.linspace(0.05, 1.95, 39):
        r, e = q * h, 1e-7 * h
        fd = (O.kernel_W(c, r + e) - O.kernel_W(c, r - e)) / (2 * e)
        assert O.kernel_dWdr(c, r) == pytest.approx(fd, rel=1e-6, abs=1e-6 * O.kernel_W(c, 0) / h)
        assert O.kernel_dWdr(c, r) < 0.0


def test_lattice_sum_approximates_the_integral():
    # a smooth unit-integral kernel summed over a lattice of spacing s (s^3 per site)
    c = cfg()
    assert abs(O.lattice_sum(c) * c.spacing ** 3 - 1.0) < 1e-3


# --------------------------------------------------------------------------
# density and equation of state
# --------------------------------------------------------------------------
def lattice(n, s, origin=(0.0, 0.0, 0.0)):
    return scenes.lattice_column((n, n, n), s, origin)


def test_rest_lattice_interior_has_rest_density():
    c = cfg()
    s = c.spacing
    x = lattice(13, s)
    centre = np.argmin(np.linalg.norm(x - x.mean(0), axis=1))
    rho, p = O.density(c, x)
    assert abs(rho[centre] - c.rho0) < 1e-12 * c.rho0
    assert p[centre] == pytest.approx(0.0, abs=1e-6)


def test_density_matches_brute_force_sum():
    c = cfg()
    rng = np.random.default_rng(1)
    x = rng.uniform(0.0, 0.25, size=(300, 3))
    rho, _ = O.density(c, x)
    info = O.derive(c)
    xf = x.astype(np.float32)
    for i in range(0, 300, 7):
        # neighbour predicate in float, as the method takes structural decisions
        d2 = fused_d2(xf - xf[i])
        nb = np.nonzero((d2 < np.float32(info.r2f)))[0]
        ref = sum(O.kernel_W(c, np.linalg.norm(x[i] - x[j])) for j in nb)
        assert rho[i] == pytest.approx(info.mass * ref, rel=1e-12)


def test_eos_speed_of_sound_and_clamp():
    c = cfg()
    assert O.eos(c, c.rho0) == 0.0
    e = 1e-6 * c.rho0
    dpdrho = (O.eos(c, c.rho0 + e) - O.eos(c, c.rho0)) / e
    assert dpdrho == pytest.approx(c.c0 ** 2, rel=1e-5)   # definition of the sound speed
    assert O.eos(c, 0.99 * c.rho0) == 0.0                    # clamped
    c2 = cfg(clamp_p=0)
    assert O.eos(c2, 0.99 * c2.rho0) < 0.0


# --------------------------------------------------------------------------
# forces
# --------------------------------------------------------------------------
def test_isolated_particle_falls_with_gravity():
    c = cfg()
    a = O.forces(c, np.array([[0.3, 0.2, 0.2]]), np.zeros((1, 3)), np.array([c.rho0]),
                 np.array([500.0]))
    assert np.allclose(a[0], c.g[:])


def test_compressed_pair_repels_symmetrically():
    c = cfg()
    x = np.array([[0.30, 0.2, 0.2], [0.31, 0.2, 0.2]])
    a = O.forces(c, x, np.zeros((2, 3)), np.full(2, 1010.0), np.full(2, 3000.0))
    g = np.array(c.g[:])
    assert (a[0] - g)[0] < 0.0 and (a[1] - g)[0] > 0.0      # pushed apart
    assert np.allclose(a[0] - g, -(a[1] - g), rtol=1e-13)


def test_term_sums_are_the_magnitudes_of_the_terms():
    """The per-particle error scale of the force comparisons: |g| alone for
    an isolated particle, |g| + |a - g| for one pair (a single term), and
    at least |a - g| (triangle inequality) with more neighbours."""
    c = cfg()
    g = np.linalg.norm(np.array(c.g[:]))
    _, ts = O.forces(c, np.array([[0.3, 0.2, 0.2]]), np.zeros((1, 3)), np.array([c.rho0]),
                     np.array([500.0]), term_sums=True)
    assert ts[0] == pytest.approx(g, rel=1e-15)
    x = np.array([[0.30, 0.2, 0.2], [0.31, 0.205, 0.2]])
    v = np.array([[0.1, 0.0, 0.0], [-0.2, 0.05, 0.0]])        # approaching: viscosity on
    a, ts = O.forces(c, x, v, np.full(2, 1010.0), np.full(2, 3000.0), term_sums=True)
    for i in range(2):
        assert ts[i] == pytest.approx(g + np.linalg.norm(a[i] - np.array(c.g[:])), rel=1e-13)
    rng = np.random.default_rng(5)
    x = rng.uniform(0.1, 0.2, size=(200, 3))
    rho, p = O.density(c, x)
    a, ts = O.forces(c, x, rng.normal(0, 0.3, (200, 3)), rho, p, term_sums=True)
    assert np.all(ts >= g + np.linalg.norm(a - np.array(c.g[:]), axis=1) * (1 - 1e-12) - g * 1e-12)


def test_momentum_is_conserved_in_a_fluid_cloud():
    c = cfg()
    rng = np.random.default_rng(2)
    x = rng.uniform(0.1, 0.3, size=(400, 3))
    v = rng.normal(0.0, 0.5, size=(400, 3))
    rho, p = O.density(c, x)
    a = O.forces(c, x, v, rho, p)
    internal = a - np.array(c.g[:])
    scale = np.abs(internal).sum()
    assert np.abs(internal.sum(0)).max() < 1e-12 * scale


def test_linear_pressure_field_gives_minus_grad_p_over_rho():
    c = cfg(clamp_p=0)
    s = c.spacing
    x = lattice(15, s)
    G = np.array([300.0, -1200.0, 700.0])                   # Pa / m
    p = 5000.0 + x @ G
    rho = np.full(x.shape[0], c.rho0)
    centre = np.argmin(np.linalg.norm(x - x.mean(0), axis=1))
    which = np.zeros(x.shape[0], np.uint8)
    which[centre] = 1
    a = O.forces(c, x, np.zeros_like(x), rho, p, which=which)[centre]
    expect = np.array(c.g[:]) - G / c.rho0
    assert np.allclose(a, expect, rtol=2e-3, atol=2e-3 * np.abs(G).max() / c.rho0)


def test_viscosity_only_damps_approach():
    c = cfg()
    x = np.array([[0.30, 0.2, 0.2], [0.31, 0.2, 0.2]])
    rho, p = np.full(2, c.rho0), np.zeros(2)
    g = np.array(c.g[:])
    same = O.forces(c, x, np.array([[1.0, 0.0, 0.0], [1.0, 0.0, 0.0]]), rho, p)
    assert np.allclose(same, g)                                # no relative motion
    apart = O.forces(c, x, np.array([[-1.0, 0.0, 0.0], [1.0, 0.0, 0.0]]), rho, p)
    assert np.allclose(apart, g)                               # receding: no viscosity
    vin = np.array([[1.0, 0.0, 0.0], [-1.0, 0.0, 0.0]])
    close = O.forces(c, x, vin, rho, p) - g
    vij = vin[0] - vin[1]
    assert np.dot(close[0] - close[1], vij) < 0.0              # relative speed decreases


def test_wall_pushes_a_compressed_particle_back():
    # a fluid slab resting on the floor; its bottom-centre particle is pushed
    # a third of a spacing towards the wall and must be pushed back up
    sc = scenes.dam_break_small()
    c = O.cfg_from_params(sc.params)
    s = c.spacing
    x = scenes.lattice_column((15, 4, 15), s, (0.0, 0.0, 0.0))
    centre = np.argmin(np.linalg.norm(x[:, [0, 2]] - x[:, [0, 2]].mean(0), axis=1) + x[:, 1])
    x[centre, 1] -= s / 3.0
    rho, p = O.density(c, x, sc.walls)
    a = O.forces(c, x, np.zeros_like(x), rho, p, sc.walls)
    assert p[centre] > 0.0 and a[centre, 1] > 0.0


# --------------------------------------------------------------------------
# integrator (Section 4.1)
# --------------------------------------------------------------------------
def test_free_fall_is_exact():
    x = np.array([[0.1, 0.5, 0.2]])
    v = np.array([[0.3, 1.0, -0.2]])
    g = np.array([[0.0, -9.81, 0.0]])
    a = g.copy()
    x0, v0 = x.copy(), v.copy()
    dt, t = 1e-3, 0.0
    for _ in range(50):
        O.serna_predict(x, v, a, dt)
        O.serna_correct(x, v, a, g.copy(), np.array([dt]))
        t += dt
    assert np.allclose(x, x0 + v0 * t + 0.5 * g * t * t, rtol=0, atol=1e-14)
    assert np.allclose(v, v0 + g * t, rtol=0, atol=1e-13)


def test_correction_is_exact_for_linearly_varying_acceleration():
    jerk, dt = 7.0, 0.01
    x, v, a = np.zeros((1, 3)), np.zeros((1, 3)), np.zeros((1, 3))
    O.serna_predict(x, v, a, dt)
    O.serna_correct(x, v, a, np.full((1, 3), jerk * dt), np.array([dt]))
    assert np.allclose(x, jerk * dt ** 3 / 6.0, rtol=1e-14)
    assert np.allclose(v, jerk * dt ** 2 / 2.0, rtol=1e-14)


def test_substeps_with_constant_acceleration_are_an_interpolation():
    rng = np.random.default_rng(3)
    x0, v0, a = rng.normal(size=(5, 3)), rng.normal(size=(5, 3)), rng.normal(size=(5, 3))
    xa, va = x0.copy(), v0.copy()
    for _ in range(8):
        O.serna_predict(xa, va, a, 1e-3)
    xb, vb = x0.copy(), v0.copy()
    O.serna_predict(xb, vb, a, 8e-3)
    assert np.allclose(xa, xb, rtol=0, atol=1e-15) and np.allclose(va, vb, rtol=0, atol=1e-15)


def test_second_order_convergence_on_an_oscillator():
    w2 = 4.0

    def run(dt, T=2.0):
        x, v = np.array([[1.0, 0.0, 0.0]]), np.zeros((1, 3))
        a = -w2 * x
        for _ in range(int(round(T / dt))):
            O.serna_predict(x, v, a, dt)
            O.serna_correct(x, v, a, -w2 * x, np.array([dt]))
        return x[0, 0]

    exact = math.cos(2.0 * 2.0)
    e1, e2 = abs(run(0.01) - exact), abs(run(0.005) - exact)
    assert 3.5 < e1 / e2 < 4.5


# --------------------------------------------------------------------------
# region determination (Section 3, 3.1, 4.2, Algorithm 1)
# --------------------------------------------------------------------------
def test_keys_place_each_particle_inside_its_block():
    c = cfg()
    info = O.derive(c)
    rng = np.random.default_rng(4)
    x = rng.uniform(c.dom_min[0], c.dom_max[1], size=(5000, 3)).astype(np.float32)
    x[:, 0] = rng.uniform(c.dom_min[0], c.dom_max[0], 5000)
    k = O.keys(c, x).astype(np.int64)
    nx, ny, nz = info.nc
    b = np.stack([k % nx, (k // nx) % ny, k // (nx * ny)], axis=1)
    e = c.block_edge
    lo = np.array(c.dom_min[:]) + b * e
    assert (k < info.nblocks).all()
    assert (x >= lo - 1e-6).all() and (x < lo + e + 1e-6).all()


def test_sort_is_the_stable_argsort():
    rng = np.random.default_rng(5)
    key = rng.integers(0, 50, size=2000).astype(np.uint32)
    perm, start = O.sort(50, key)
    assert np.array_equal(perm, np.argsort(key, kind="stable"))
    assert np.array_equal(start, np.concatenate([[0], np.cumsum(np.bincount(key, minlength=50))]))


def test_neighbours_match_brute_force():
    sc = scenes.dam_break_small()
    c = O.cfg_from_params(sc.params)
    info = O.derive(c)
    rng = np.random.default_rng(6)
    x = rng.uniform(0.0, 0.3, size=(700, 3)).astype(np.float32)
    w = sc.walls.astype(np.float32)
    st, nbr, nnb = O.neighbors(c, x, w)
    assert st == 0
    for i in range(0, 700, 11):
        d2 = fused_d2(x - x[i])
        f = set(np.nonzero(d2 < info.r2f)[0].tolist()) - {i}
        d2w = fused_d2(w - x[i])
        wl = set((np.nonzero(d2w < info.r2f)[0] | O.WALL_BIT).tolist())
        got = nbr[i, :nnb[i]].tolist()
        assert len(got) == len(set(got))
        assert set(got) == f | wl


def test_level_thresholds_follow_the_paper_constants():
    gold = json.load(open(GOLDEN))
    c = cfg(mode="rts", level_cap=3)
    info = O.derive(c)
    assert c.lambda_v == gold["lambda_v_max"] and c.lambda_f == gold["lambda_f_max"]
    assert c.alpha_rts == gold["alpha_wcsph"]
    dt, r = info.dt_base, c.r_crit
    assert math.isinf(info.TV[0])
    for l in (1, 2, 3):
        vmax = gold["alpha_wcsph"] * gold["beta"][str(l + 1)] * r / (2 ** l * dt)
        assert info.TV[l] == pytest.approx(vmax * vmax, rel=1e-6)
        amax = gold["lambda_f_max"] ** 2 * r / (2 ** l * dt) ** 2
        assert info.TA[l] == pytest.approx(amax * amax, rel=1e-6)


def test_block_level_is_the_largest_admissible():
    c = cfg(mode="rts", level_cap=3)
    info = O.derive(c)
    vs = [math.sqrt(info.TV[1]) * 1.01, math.sqrt(info.TV[1]) * 0.99,
          math.sqrt(info.TV[2]) * 0.99, math.sqrt(info.TV[3]) * 0.99]
    expect = [0, 1, 2, 3]
    key = np.arange(4, dtype=np.uint32) * 3
    vel = np.zeros((4, 3), np.float32)
    vel[:, 0] = vs
    lv = O.block_levels(c, key, vel, np.zeros((4, 3), np.float32))
    assert list(lv[key]) == expect
    assert (np.delete(lv, key) == O.EMPTY_BLOCK).all()
    acc = np.zeros((4, 3), np.float32)
    acc[:, 1] = math.sqrt(info.TA[1]) * 1.01                 # Eq. 2 now forbids level >= 1
    lv2 = O.block_levels(c, key, np.zeros((4, 3), np.float32), acc)
    assert (lv2[key] == 0).all()


def test_rmin_takes_the_smaller_neighbour_level_once():
    c = cfg()
    info = O.derive(c)
    nx, ny, nz = info.nc
    lvl = np.full(info.nblocks, 3, np.uint8)
    k0 = 4 + nx * (4 + ny * 4)
    lvl[k0] = 0
    lvl[1 + nx * (1 + ny * 1)] = O.EMPTY_BLOCK
    out = O.rmin(c, lvl)
    for dz in range(-2, 3):
        for dy in range(-2, 3):
            for dx in range(-2, 3):
                k = (4 + dx) + nx * ((4 + dy) + ny * (4 + dz))
                inner = max(abs(dx), abs(dy), abs(dz)) <= 1
                assert out[k] == (0 if inner else 3)
    assert out[1 + nx * (1 + ny * 1)] == O.EMPTY_BLOCK


def test_particles_at_level_l_are_active_every_2_to_the_l_steps():
    key = np.zeros(4, np.uint32)
    for l in range(4):
        blk = np.array([l], np.uint8)
        level = np.full(4, 0xF, np.int32)
        val = np.zeros(4, np.int32)
        active = []
        for step in range(40):
            level, val, comp = O.flags(key, blk, level, val)
            active.append(bool(comp[0]))
        assert [k for k, a in enumerate(active) if a] == list(range(0, 40, 2 ** l))


def test_preemption_when_the_block_level_changes():
    key = np.zeros(1, np.uint32)
    level, val, comp = O.flags(key, np.array([3], np.uint8), np.full(1, 0xF, np.int32),
                               np.zeros(1, np.int32))
    assert comp[0] == 1 and val[0] == 8
    level, val, comp = O.flags(key, np.array([3], np.uint8), level, val)
    assert comp[0] == 0
    level, val, comp = O.flags(key, np.array([1], np.uint8), level, val)
    assert comp[0] == 1 and level[0] == 1 and val[0] == 2


@pytest.mark.parametrize("step,level,validity", [
    (0, 3, 8), (13, 3, 3), (16, 3, 8), (23, 3, 1), (13, 2, 3), (14, 2, 2), (15, 1, 1),
    (16, 1, 2), (7, 0, 1), (101, 0, 1)])
def test_phase_aligned_validity_runs_to_the_next_multiple(step, level, validity):
    """Phase alignment: a particle that takes level l at base step k is next
    due at the first multiple of 2^l after k (hand-computed table)."""
    key = np.zeros(1, np.uint32)
    lv, val, comp = O.flags(key, np.array([level], np.uint8), np.full(1, 0xF, np.int32),
                            np.zeros(1, np.int32), step=step, phase_align=1)
    assert comp[0] == 1 and lv[0] == level and val[0] == validity
    # Algorithm 1 as printed: 2^l steps from now, whatever the step index
    lv, val, comp = O.flags(key, np.array([level], np.uint8), np.full(1, 0xF, np.int32),
                            np.zeros(1, np.int32), step=step, phase_align=0)
    assert val[0] == 2 ** level


def test_phase_aligned_particles_of_a_level_update_together():
    """Particles taking level 3 at different steps (their block's level
    changes at staggered times) end up due on the same steps, the multiples
    of 8, and no step is longer than 8 base steps."""
    key = np.arange(4, dtype=np.uint32)
    level = np.full(4, 0xF, np.int32)
    val = np.zeros(4, np.int32)
    blk = np.zeros(4, np.uint8)
    due = {i: [] for i in range(4)}
    last = np.zeros(4, np.int64)
    for step in range(48):
        blk = np.array([3 if step >= s else 0 for s in (0, 3, 5, 11)], np.uint8)
        level, val, comp = O.flags(key, blk, level, val, step=step, phase_align=1)
        for i in range(4):
            if comp[i]:
                assert step == 0 or step - last[i] <= 2 ** 3
                last[i] = step
                due[i].append(step)
    for i in range(4):
        late = [k for k in due[i] if k >= 16]
        assert late == [16, 24, 32, 40], (i, due[i])


def test_phase_aligned_run_computes_exactly_on_multiples_or_level_changes():
    """A developed RTS run with phase alignment: at every base step k a
    particle computes iff its level changed at k or k is a multiple of
    2^level; with level cap 0 the run is global stepping bit for bit."""
    sc = scenes.dam_break_column(counts=(10, 14, 8), spacing=0.02, box=(0.6, 0.4, 0.3),
                                 c0=scenes.sound_speed_for_column(0.28, factor=10.0))
    a = O.WCSPH(sc.params, sc.pos, walls=sc.walls, mode="rts", phase_align=1)
    prev = a.level.copy()
    seen_levels = set()
    for k in range(60):
        a.step(1)
        lv = a.level
        seen_levels |= set(np.unique(lv).tolist())
        want = (lv != prev) | (k % (1 << lv) == 0)
        assert np.array_equal(a.compute.astype(bool), want), f"step {k}"
        prev = lv.copy()
    assert len(seen_levels) >= 2
    b = O.WCSPH(sc.params, sc.pos, walls=sc.walls, mode="rts", level_cap=0, phase_align=1)
    g = O.WCSPH(sc.params, sc.pos, walls=sc.walls, mode="global_fixed")
    b.step(12)
    g.step(12)
    assert np.array_equal(b.x, g.x) and np.array_equal(b.v, g.v)


def test_rts_with_every_block_at_level_zero_is_global_stepping():
    sc = scenes.dam_break_column(counts=(10, 14, 8), spacing=0.02, box=(0.6, 0.4, 0.3))
    a = O.WCSPH(sc.params, sc.pos, walls=sc.walls, mode="rts", level_cap=0)
    b = O.WCSPH(sc.params, sc.pos, walls=sc.walls, mode="global_fixed")
    a.step(15)
    b.step(15)
    assert np.array_equal(a.x, b.x) and np.array_equal(a.v, b.v)


def test_rts_skips_work_but_stays_close_to_global():
    sc = scenes.dam_break_column(counts=(10, 14, 8), spacing=0.02, box=(0.6, 0.4, 0.3))
    a = O.WCSPH(sc.params, sc.pos, walls=sc.walls, mode="rts")
    b = O.WCSPH(sc.params, sc.pos, walls=sc.walls, mode="global_fixed")
    a.step(40)
    b.step(40)
    assert sum(h["n_active"] for h in a.history) < 0.8 * sum(h["n_active"] for h in b.history)
    assert np.abs(a.x - b.x).max() < 0.05 * sc.params["spacing"]
