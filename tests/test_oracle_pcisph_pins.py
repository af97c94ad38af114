"""Pins of the CPU oracle's PCISPH part against mathematics, brute force and
the constraints the paper states (no GPU).

Section "Regional Time Stepping with PCISPH": regions 1-4 from Eq. 2-3 with
alpha = 1, dilation of regions 1 and 2, observed blocks, the correction
schedule, asynchronous neighbourhoods on a grid of edge 1.1 r kept for a
major step, and the standard PCISPH pressure coefficient delta.
"""
import itertools

import numpy as np
import pytest

import oracle as O
from paper_2009_14514_amd import scenes


def pscene(**kw):
    return scenes.pcisph_dam_break_small(**kw)


def pcfg(**over):
    return O.cfg_from_params(pscene().params, **over)


def block_coords(info, keys):
    nx, ny = info.nc[0], info.nc[1]
    keys = np.asarray(keys, np.int64)
    return np.stack([keys % nx, (keys // nx) % ny, keys // (nx * ny)], axis=1)


# --------------------------------------------------------------------------
# a19: delta
# --------------------------------------------------------------------------
def test_delta_cancels_a_density_error_on_the_prototype_lattice():
    """One pressure p = delta * err applied by the centre particle of a full
    rest lattice moves its neighbours (by dt^2 times the pressure force of
    that pressure, standard PCISPH's derivation) so that the recomputed
    kernel sum of the centre drops by err to first order."""
    c = pcfg()
    info = O.derive(c)
    s, r, m, rho0, dt = c.spacing, c.support, info.mass, c.rho0, info.dt_base
    K = int(np.ceil(r / s)) + 1
    offs = np.array([v for v in itertools.product(range(-K, K + 1), repeat=3)
                     if v != (0, 0, 0)], np.float64) * s
    d = np.linalg.norm(offs, axis=1)
    offs, d = offs[d < r], d[d < r]

    def rho_centre(pos):
        dist = np.linalg.norm(pos, axis=1)
        return m * (O.kernel_W(c, 0.0) + sum(O.kernel_W(c, x) for x in dist))

    assert rho_centre(offs) == pytest.approx(rho0, rel=1e-12)
    for err in (1e-4, -1e-4, 5e-4):
        p = info.delta * err
        # gradient of W at x_centre - x_j = -offs_j
        dwdr = np.array([O.kernel_dWdr(c, x) for x in d])
        grad = (dwdr / d)[:, None] * (-offs)
        # reaction on neighbour j from the centre's pressure (neighbours at p, rho0):
        # F_j = m^2 (2 p / rho0^2) gradW_ij ; dx_j = dt^2 F_j / m
        dx = dt * dt * m * (2.0 * p / rho0 ** 2) * grad
        # the centre itself does not move: sum_j gradW_ij = 0 on the lattice
        assert np.abs(grad.sum(axis=0)).max() < 1e-9 * np.abs(grad).sum()
        change = rho_centre(offs + dx) - rho0
        assert change == pytest.approx(-err, rel=2e-2, abs=0)


def test_delta_scales_with_inverse_step_squared():
    d1 = O.pci_delta(pcfg(dt_base=1e-3))
    d2 = O.pci_delta(pcfg(dt_base=2e-3))
    assert d1 > 0 and d2 == pytest.approx(d1 / 4.0, rel=1e-12)


# --------------------------------------------------------------------------
# a13: regions
# --------------------------------------------------------------------------
def test_region_thresholds_use_multiples_of_the_base_step_and_alpha_one():
    c = pcfg()
    info = O.derive(c)
    r, dt = c.r_crit, info.dt_base
    betas = [np.inf, 0.4, 0.08, 0.016]
    for k in range(4):
        n = k + 1
        v = np.inf if np.isinf(betas[k]) else 1.0 * betas[k] * r / (n * dt)
        a = 0.25 ** 2 * r / (n * dt) ** 2
        assert info.TV[k] == np.float32(v * v)
        assert info.TA[k] == np.float32(a * a)


def hand_grid(c, fill=3):
    info = O.derive(c)
    lvl = np.full(info.nblocks, fill, np.uint8)
    return info, lvl


def chebyshev(info, a, b):
    ca, cb = block_coords(info, a), block_coords(info, b)
    return np.abs(ca[:, None, :] - cb[None, :, :]).max(axis=2)


def test_dilation_grows_a_level_by_chebyshev_layers():
    c = pcfg()
    info, lvl = hand_grid(c)
    nb = int(info.nblocks)
    rng = np.random.default_rng(1)
    empty = rng.random(nb) < 0.2
    lvl[empty] = O.EMPTY_BLOCK
    seeds = rng.choice(np.nonzero(~empty)[0], 2, replace=False)
    lvl[seeds] = 0
    for layers in (1, 2, 4):
        out = O.pci_dilate(c, lvl, 0, layers)
        dist = chebyshev(info, np.arange(nb), seeds).min(axis=1)
        want = lvl.copy()
        want[(dist <= layers) & ~empty] = 0
        assert np.array_equal(out, want)


def test_region_two_dilates_after_region_one():
    c = pcfg()
    info, lvl = hand_grid(c)
    nb = int(info.nblocks)
    lvl[5] = 1
    lvl[nb - 3] = 0
    raw = lvl.copy()
    t1 = O.pci_dilate(c, raw, 0, 4)
    t2 = O.pci_dilate(c, t1, 1, 4)
    d1 = chebyshev(info, np.arange(nb), [nb - 3])[:, 0]
    d2 = chebyshev(info, np.arange(nb), np.nonzero(t1 == 1)[0]).min(axis=1)
    want = np.full(nb, 3, np.uint8)
    want[d2 <= 4] = 1
    want[d1 <= 4] = 0
    assert np.array_equal(t2, want)


def test_observed_blocks_border_a_smaller_region():
    c = pcfg()
    info, lvl = hand_grid(c)
    nb = int(info.nblocks)
    rng = np.random.default_rng(7)
    lvl = rng.integers(0, 4, nb).astype(np.uint8)
    lvl[rng.random(nb) < 0.15] = O.EMPTY_BLOCK
    ob = O.pci_observed(c, lvl)
    dist = chebyshev(info, np.arange(nb), np.arange(nb))
    want = np.zeros(nb, np.uint8)
    for b in range(nb):
        if lvl[b] == O.EMPTY_BLOCK:
            continue
        nbrs = np.nonzero(dist[b] <= 1)[0]
        want[b] = np.any(lvl[nbrs] < lvl[b])
    assert np.array_equal(ob, want)


def test_regions_of_a_resting_scene_are_the_slowest():
    sc = pscene()
    c = O.cfg_from_params(sc.params)
    key = O.keys(c, sc.pos.astype(np.float32))
    z = np.zeros_like(sc.pos, dtype=np.float32)
    raw, lvl, ob = O.pci_regions(c, key, z, z)
    occ = np.unique(key)
    assert np.all(raw[occ] == 3) and np.all(lvl[occ] == 3) and not ob.any()
    # one fast particle makes its block region 1 and, through the dilation,
    # every occupied block within four layers
    v = z.copy()
    v[0] = (10.0, 0.0, 0.0)     # above the region-2 bound of 8 m/s
    raw, lvl, ob = O.pci_regions(c, key, v, z)
    info = O.derive(c)
    assert raw[key[0]] == 0
    dist = chebyshev(info, occ, [key[0]])[:, 0]
    assert np.all(lvl[occ[dist <= 4]] == 0)


# --------------------------------------------------------------------------
# a17: the schedule
# --------------------------------------------------------------------------
def test_schedule_meets_the_stated_constraints():
    """Every region at least once per minor step, all regions twice in the
    first minor step, region 1 three times per minor step, region 2 three
    times per two minor steps, slower regions no more than faster ones, and
    every region at least three times within its own step."""
    rows = lambda col, n: sum((O.pci_turn(col, row) >> (n - 1)) & 1 for row in (1, 2, 3))
    for col in range(4):
        for n in range(1, 5):
            assert rows(col, n) >= 1
    for n in range(1, 5):
        assert rows(0, n) >= 2
    for col in range(4):
        assert rows(col, 1) == 3
    assert rows(0, 2) + rows(1, 2) == 3 and rows(2, 2) + rows(3, 2) == 3
    total = [sum(rows(col, n) for col in range(4)) for n in range(1, 5)]
    assert total == sorted(total, reverse=True)
    for n in range(1, 5):
        assert sum(rows(col, n) for col in range(min(n, 4))) >= 3
    assert O.pci_turn(0, 4) == 0 and O.pci_turn(4, 1) == 0


# --------------------------------------------------------------------------
# a14: lists on the stored grid
# --------------------------------------------------------------------------
def fused_d2(d):
    d = np.asarray(d, np.float32).astype(np.float64)
    xx = (d[..., 0] * d[..., 0]).astype(np.float32).astype(np.float64)
    s = (d[..., 1] * d[..., 1] + xx).astype(np.float32).astype(np.float64)
    return (d[..., 2] * d[..., 2] + s).astype(np.float32)


@pytest.mark.parametrize("rings", [1, 2])
def test_lists_match_brute_force_with_a_stale_grid(rings):
    sc = pscene(counts=(6, 10, 5))
    c = O.cfg_from_params(sc.params)
    info = O.derive(c)
    x0 = sc.pos.astype(np.float32)
    key0 = O.keys(c, x0)
    perm, start = O.sort(info.nblocks, key0)
    xs = x0[perm]
    key = key0[perm]
    # particles move after the grid was built
    rng = np.random.default_rng(3)
    moved = (xs + rng.normal(0, 0.3 * c.block_edge, xs.shape)).astype(np.float32)
    wx, wstart, _ = O.sorted_walls(c, sc.walls)
    wx32 = wx.astype(np.float32)
    wkey = O.keys(c, wx32)
    st, nbr, nnb = O.pci_lists(c, moved, start, key, wx32, wstart,
                               rings=np.full(len(xs), rings, np.uint8), cap=1024)
    assert st == 0
    r2l = np.float32(c.block_edge ** 2)
    bc, wc = block_coords(info, key), block_coords(info, wkey)
    for i in range(0, len(xs), 7):
        near_blocks = np.abs(bc - bc[i]).max(axis=1) <= rings
        d2 = fused_d2(moved - moved[i])
        fl = np.nonzero(near_blocks & (d2 < r2l) & (np.arange(len(xs)) != i))[0]
        wnear = np.abs(wc - bc[i]).max(axis=1) <= rings
        wd2 = fused_d2(wx32 - moved[i])
        wl = np.nonzero(wnear & (wd2 < r2l))[0]
        want = np.concatenate([fl, wl | O.WALL_BIT]).astype(np.uint32)
        assert np.array_equal(nbr[i, :nnb[i]], want)


# --------------------------------------------------------------------------
# physics pieces
# --------------------------------------------------------------------------
def lattice_block(c, n=9):
    s = c.spacing
    g = np.stack(np.meshgrid(*[np.arange(n) * s] * 3, indexing="ij"), axis=-1).reshape(-1, 3)
    return g + 0.37


def all_lists(c, x, walls=None):
    info = O.derive(c)
    x32 = x.astype(np.float32)
    key0 = O.keys(c, x32)
    perm, start = O.sort(info.nblocks, key0)
    w = np.zeros((0, 3)) if walls is None else walls
    wx, wstart, _ = O.sorted_walls(c, w)
    st, nbr, nnb = O.pci_lists(c, x32[perm], start, key0[perm], wx.astype(np.float32), wstart,
                               cap=c.nbr_cap)
    assert st == 0
    return x[perm], nbr, nnb, wx


def test_rest_lattice_interior_has_rest_density():
    c = pcfg(nbr_cap=1024)
    x, nbr, nnb, wx = all_lists(c, lattice_block(c))
    rho = O.pci_density(c, x, wx, nbr, nnb)
    centre = np.argmin(np.linalg.norm(x - x.mean(axis=0), axis=1))
    assert rho[centre] == pytest.approx(c.rho0, rel=1e-12)


def test_pressure_forces_conserve_momentum_and_vanish_for_uniform_pressure():
    c = pcfg(nbr_cap=1024)
    rng = np.random.default_rng(5)
    x = lattice_block(c, 7) + rng.normal(0, 0.1 * c.spacing, (343, 3))
    x, nbr, nnb, wx = all_lists(c, x)
    rho = O.pci_density(c, x, wx, nbr, nnb)
    p = rng.uniform(0, 500, len(x))
    fp = O.pci_pressure_force(c, x, wx, p, rho, nbr, nnb)
    scale = np.abs(fp).sum()
    assert np.abs(fp.sum(axis=0)).max() < 1e-12 * scale
    # interior of a rest lattice with uniform pressure: no force
    x2, nbr2, nnb2, wx2 = all_lists(c, lattice_block(c))
    rho2 = np.full(len(x2), c.rho0)
    fp2 = O.pci_pressure_force(c, x2, wx2, np.full(len(x2), 1e3), rho2, nbr2, nnb2)
    centre = np.argmin(np.linalg.norm(x2 - x2.mean(axis=0), axis=1))
    assert np.abs(fp2[centre]).max() < 1e-9 * np.abs(fp2).max()


def test_pressure_force_term_sums_bound_the_force():
    """The per-particle error scale of the pressure-force comparison is the
    sum of the pair terms' magnitudes: it equals |F^p| for a lone pair and
    bounds it (triangle inequality) in a cloud."""
    c = pcfg(nbr_cap=1024)
    x = np.array([[0.3, 0.2, 0.15], [0.3 + 0.7 * c.spacing, 0.2 + 0.6 * c.spacing, 0.15]])
    x, nbr, nnb, wx = all_lists(c, x)
    assert list(nnb) == [1, 1]
    fp, ts = O.pci_pressure_force(c, x, wx, np.array([300.0, 800.0]), np.array([1001.0, 1003.0]),
                                  nbr, nnb, term_sums=True)
    assert np.allclose(ts, np.linalg.norm(fp, axis=1), rtol=1e-13)
    rng = np.random.default_rng(5)
    x = lattice_block(c, 7) + rng.normal(0, 0.1 * c.spacing, (343, 3))
    x, nbr, nnb, wx = all_lists(c, x)
    rho = O.pci_density(c, x, wx, nbr, nnb)
    fp, ts = O.pci_pressure_force(c, x, wx, rng.uniform(0, 500, len(x)), rho, nbr, nnb,
                                  term_sums=True)
    assert np.all(ts >= np.linalg.norm(fp, axis=1) * (1 - 1e-12))


def test_nonpressure_is_gravity_plus_momentum_free_viscosity():
    c = pcfg(nbr_cap=1024)
    rng = np.random.default_rng(9)
    x = lattice_block(c, 6) + rng.normal(0, 0.05 * c.spacing, (216, 3))
    x, nbr, nnb, wx = all_lists(c, x)
    v = rng.normal(0, 0.5, x.shape)
    f = O.pci_nonpressure(c, x, v, wx, nbr, nnb)
    visc = f - np.asarray(c.g)[None, :]
    assert np.abs(visc.sum(axis=0)).max() < 1e-12 * np.abs(visc).sum()
    f0 = O.pci_nonpressure(c, x, np.zeros_like(v) + 0.3, wx, nbr, nnb)
    assert np.allclose(f0, np.asarray(c.g)[None, :], rtol=0, atol=1e-12)


# --------------------------------------------------------------------------
# whole steps
# --------------------------------------------------------------------------
def test_all_region_one_is_standard_pcisph_when_the_schedule_suffices():
    """RTS with every block capped at region 1 takes every particle in rows
    1-3 of every minor step; with lists that hold the same neighbour sets it
    is standard PCISPH (grid rebuilt every step) up to summation order."""
    sc = pscene(counts=(6, 12, 6))
    a = O.PCISPH(sc.params, sc.pos, walls=sc.walls, level_cap=0)
    b = O.PCISPH(sc.params, sc.pos, walls=sc.walls, mode=1)
    for k in range(6):
        a.step()
        b.step()
        ha, hb = a.history[-1], b.history[-1]
        assert ha["iters"] == hb["iters"]
        xa = a.in_caller_order(a.x)
        xb = b.in_caller_order(b.x)
        assert np.abs(xa - xb).max() < 1e-9 * sc.params["spacing"]


def test_resting_column_stays_within_the_error_bound():
    """A column filling its box settles: every minor step ends below the
    allowed compression and nothing moves fast."""
    sc = scenes.pcisph_column()
    sim = O.PCISPH(sc.params, sc.pos, walls=sc.walls)
    sim.step(12)
    for h in sim.history:
        assert h["iters"] >= 3
        assert h["errmax"] < sc.params["eta"] or h["iters"] == sc.params["it_max"]
    assert max(h["errmax"] for h in sim.history) < sc.params["eta"]
    # settling of the jitter only: slower than a fall through one spacing
    assert np.linalg.norm(sim.v, axis=1).max() < np.sqrt(2 * 9.81 * sc.params["spacing"])


def test_two_layer_variant_searches_region_two_with_two_layers():
    """With two_ring_levels = 2 a minor step builds region-2 lists over two
    block layers of the stored grid (brute force on the same snapshot)."""
    sc = pscene(v0=1.5)
    sim = O.PCISPH(sc.params, sc.pos, vel=sc.vel, walls=sc.walls, two_ring_levels=2)
    sim.major_begin()
    assert np.all(sim.region == 2)
    x32 = sim.x.astype(np.float32)
    sim.step()
    st, nbr, nnb = O.pci_lists(sim.cfg, x32, sim.cell_start, sim.key, sim.wx.astype(np.float32),
                               sim.wcell_start, rings=np.full(sc.n, 2, np.uint8))
    assert st == 0
    assert np.array_equal(sim.nnb[:sc.n], nnb)
    assert np.array_equal(sim.nbr[:sc.n], nbr)
