"""Pins of the oracle's differentiable WCSPH substeps and their adjoint (no
GPU): central finite differences on the oracle's own forward run, and the
closed form of an isolated particle under symplectic Euler."""
import numpy as np
import pytest

import oracle as O
from paper_2009_14514_amd import scenes


@pytest.fixture(scope="module")
def setup():
    sc = scenes.diff_scene()
    c = O.cfg_from_params(sc.params)
    info = O.derive(c)
    B, alpha = info.B, sc.params["visc_alpha"]
    dt, ns = sc.params["diff_dt"], sc.params["diff_substeps"]
    xT, _ = O.diff_run(c, sc.pos, sc.vel, sc.walls, B, alpha, dt, ns)
    xhat = xT + scenes.target_noise(sc.n, sc.params["target_sigma"])
    grads = O.diff_grad(c, sc.pos, sc.vel, sc.walls, B, alpha, dt, ns, xhat)
    return sc, c, B, alpha, dt, ns, xhat, grads


def loss_of(sc, c, dt, ns, xhat, x0=None, v0=None, B=None, alpha=None):
    x, _ = O.diff_run(c, sc.pos if x0 is None else x0, sc.vel if v0 is None else v0, sc.walls,
                      B, alpha, dt, ns)
    return ((x - xhat) ** 2).sum() / sc.n


def test_adjoint_matches_central_differences(setup):
    sc, c, B, alpha, dt, ns, xhat, (L, gx, gv, gB, ga) = setup
    rng = np.random.default_rng(11)
    eps = 1e-6
    fd_v, ad_v = [], []
    for _ in range(12):
        i, d = rng.integers(sc.n), rng.integers(3)
        vp, vm = sc.vel.copy(), sc.vel.copy()
        vp[i, d] += eps
        vm[i, d] -= eps
        fd_v.append((loss_of(sc, c, dt, ns, xhat, v0=vp, B=B, alpha=alpha) -
                     loss_of(sc, c, dt, ns, xhat, v0=vm, B=B, alpha=alpha)) / (2 * eps))
        ad_v.append(gv[i, d])
    fd_v, ad_v = np.array(fd_v), np.array(ad_v)
    assert np.linalg.norm(fd_v - ad_v) <= 1e-6 * np.linalg.norm(ad_v)
    fd_x, ad_x = [], []
    for _ in range(4):
        i, d = rng.integers(sc.n), rng.integers(3)
        xp, xm = sc.pos.copy(), sc.pos.copy()
        xp[i, d] += eps
        xm[i, d] -= eps
        fd_x.append((loss_of(sc, c, dt, ns, xhat, x0=xp, B=B, alpha=alpha) -
                     loss_of(sc, c, dt, ns, xhat, x0=xm, B=B, alpha=alpha)) / (2 * eps))
        ad_x.append(gx[i, d])
    fd_x, ad_x = np.array(fd_x), np.array(ad_x)
    assert np.linalg.norm(fd_x - ad_x) <= 1e-6 * np.linalg.norm(ad_x)
    eB, ea = 1e-6 * B, 1e-6 * alpha
    fdB = (loss_of(sc, c, dt, ns, xhat, B=B + eB, alpha=alpha) -
           loss_of(sc, c, dt, ns, xhat, B=B - eB, alpha=alpha)) / (2 * eB)
    fda = (loss_of(sc, c, dt, ns, xhat, B=B, alpha=alpha + ea) -
           loss_of(sc, c, dt, ns, xhat, B=B, alpha=alpha - ea)) / (2 * ea)
    assert fdB == pytest.approx(gB, rel=1e-6)
    assert fda == pytest.approx(ga, rel=1e-6)


def test_directional_derivative_over_all_velocities(setup):
    sc, c, B, alpha, dt, ns, xhat, (L, gx, gv, gB, ga) = setup
    d = np.random.default_rng(5).normal(size=sc.vel.shape)
    eps = 1e-6
    fd = (loss_of(sc, c, dt, ns, xhat, v0=sc.vel + eps * d, B=B, alpha=alpha) -
          loss_of(sc, c, dt, ns, xhat, v0=sc.vel - eps * d, B=B, alpha=alpha)) / (2 * eps)
    assert fd == pytest.approx((gv * d).sum(), rel=1e-6)


def test_isolated_particle_follows_symplectic_euler_in_closed_form():
    sc = scenes.diff_scene()
    c = O.cfg_from_params(sc.params)
    x0 = np.array([[0.15, 0.2, 0.15]])
    v0 = np.array([[0.3, -0.1, 0.2]])
    dt, n = 1e-4, 16
    g = np.asarray(sc.params["gravity"])
    xT, vT = O.diff_run(c, x0, v0, np.zeros((0, 3)), 1e5, 0.05, dt, n)
    assert np.allclose(vT, v0 + n * dt * g, rtol=0, atol=1e-15)
    assert np.allclose(xT, x0 + n * dt * v0 + g * dt * dt * n * (n + 1) / 2, rtol=0, atol=1e-15)
    xhat = xT + 0.01
    L, gx, gv, gB, ga = O.diff_grad(c, x0, v0, np.zeros((0, 3)), 1e5, 0.05, dt, n, xhat)
    assert L == pytest.approx(3 * 1e-4, rel=1e-9)
    assert np.allclose(gv, 2 * (xT - xhat) * n * dt, rtol=1e-12)
    assert np.allclose(gx, 2 * (xT - xhat), rtol=1e-12)
    assert gB == 0.0 and ga == 0.0
