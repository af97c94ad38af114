"""GPU parity of the differentiable WCSPH substeps and their adjoint.

The forward run and the gradients of L = mean |x(T) - xhat|^2 (initial
positions and velocities, Tait stiffness, viscosity alpha) are compared
with the FP64 oracle on the 512-particle scene; checkpoint spacing must
not change any bit; the autograd wrapper must return the same gradients.
A dense cluster, whose block neighbourhoods exceed the LDS staging of the
list build, takes the path that reads candidates from memory; a lone
particle follows symplectic Euler's closed form, forward and adjoint.
"""
import numpy as np
import pytest

import oracle
from paper_2009_14514_amd import scenes

pytestmark = pytest.mark.gpu


def torch():
    import torch as t
    return t


@pytest.fixture(scope="module")
def case():
    from paper_2009_14514_amd.diff import DiffRollout
    T = torch()
    sc = scenes.diff_scene()
    model = DiffRollout(sc, n_sub=16, ckpt_every=4)
    x0 = T.tensor(sc.pos, dtype=T.float32, device="cuda")
    v0 = T.tensor(sc.vel, dtype=T.float32, device="cuda")
    cfg = oracle.cfg_from_params(sc.params)
    x0h, v0h = x0.cpu().numpy().astype(np.float64), v0.cpu().numpy().astype(np.float64)
    B, alpha = model.B0, model.alpha0
    xT_ref, _ = oracle.diff_run(cfg, x0h, v0h, sc.walls, B, alpha, model.dt, 16)
    xhat = xT_ref + scenes.target_noise(sc.n, sc.params["target_sigma"])
    yield sc, model, x0, v0, cfg, x0h, v0h, B, alpha, xhat
    model.close()


def test_forward_matches_the_oracle(case):
    sc, model, x0, v0, cfg, x0h, v0h, B, alpha, xhat = case
    xT, vT = model.forward(x0, v0, B, alpha)
    xr, vr = oracle.diff_run(cfg, x0h, v0h, sc.walls, B, alpha, model.dt, 16)
    assert np.abs(xT.cpu().numpy() - xr).max() <= 1e-4 * sc.params["spacing"]
    assert np.linalg.norm(vT.cpu().numpy() - vr) <= 1e-4 * np.linalg.norm(vr)


def test_gradients_match_the_oracle_adjoint(case):
    sc, model, x0, v0, cfg, x0h, v0h, B, alpha, xhat = case
    T = torch()
    xT, _ = model.forward(x0, v0, B, alpha)
    g = 2.0 * (xT - T.tensor(xhat, dtype=T.float32, device="cuda")) / sc.n
    gx, gv, gB, ga = model.backward(g)
    L, rgx, rgv, rgB, rga = oracle.diff_grad(cfg, x0h, v0h, sc.walls, B, alpha, model.dt, 16, xhat)
    gv, gx = gv.cpu().numpy().astype(np.float64), gx.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(gv - rgv) <= 1e-3 * np.linalg.norm(rgv)
    assert np.linalg.norm(gx - rgx) <= 1e-3 * np.linalg.norm(rgx)
    assert gB == pytest.approx(rgB, rel=1e-3)
    assert ga == pytest.approx(rga, rel=1e-3)


def test_checkpoint_spacing_changes_no_bit(case):
    from paper_2009_14514_amd.diff import DiffRollout
    sc, model, x0, v0, cfg, x0h, v0h, B, alpha, xhat = case
    T = torch()
    xhat_t = T.tensor(xhat, dtype=T.float32, device="cuda")
    out = []
    for every in (1, 4, 16, 5):
        m = DiffRollout(sc, n_sub=16, ckpt_every=every)
        xT, _ = m.forward(x0, v0, B, alpha)
        gx, gv, gB, ga = m.backward(2.0 * (xT - xhat_t) / sc.n)
        out.append((xT.cpu().numpy(), gv.cpu().numpy(), gx.cpu().numpy(), gB, ga))
        m.close()
    for o in out[1:]:
        assert np.array_equal(o[0], out[0][0]) and np.array_equal(o[1], out[0][1])
        assert np.array_equal(o[2], out[0][2]) and o[3] == out[0][3] and o[4] == out[0][4]


def test_autograd_function_returns_the_adjoint(case):
    from paper_2009_14514_amd.diff import rollout_function
    sc, model, x0, v0, cfg, x0h, v0h, B, alpha, xhat = case
    T = torch()
    f = rollout_function()
    v = v0.clone().requires_grad_(True)
    Bt = T.tensor(B, dtype=T.float64, requires_grad=True)
    at = T.tensor(alpha, dtype=T.float64, requires_grad=True)
    xT = f.apply(x0, v, Bt, at, model)
    loss = ((xT - T.tensor(xhat, dtype=T.float32, device="cuda")) ** 2).sum() / sc.n
    loss.backward()
    L, rgx, rgv, rgB, rga = oracle.diff_grad(cfg, x0h, v0h, sc.walls, B, alpha, model.dt, 16, xhat)
    assert loss.item() == pytest.approx(L, rel=1e-3)
    assert np.linalg.norm(v.grad.cpu().numpy() - rgv) <= 1e-3 * np.linalg.norm(rgv)
    assert Bt.grad.item() == pytest.approx(rgB, rel=1e-3)
    assert at.grad.item() == pytest.approx(rga, rel=1e-3)


def test_second_forward_before_backward_is_refused(case):
    """One rollout keeps one tape: a backward whose forward was followed by
    another forward on the same rollout must not run on the wrong tape."""
    from paper_2009_14514_amd.diff import rollout_function
    sc, model, x0, v0, cfg, x0h, v0h, B, alpha, xhat = case
    T = torch()
    f = rollout_function()
    v = v0.clone().requires_grad_(True)
    Bt = T.tensor(B, dtype=T.float64, requires_grad=True)
    at = T.tensor(alpha, dtype=T.float64, requires_grad=True)
    first = f.apply(x0, v, Bt, at, model)
    second = f.apply(x0, v * 1.01, Bt, at, model)
    with pytest.raises(RuntimeError, match="tape"):
        first.sum().backward()
    second.sum().backward()        # the latest forward still differentiates
    assert v.grad is not None


def test_101k_scene_directional_derivatives_match_the_oracle_adjoint():
    """The 101,306-particle scene of the benchmark (37 x 74 x 37, 16
    substeps, checkpoints every 4): eight directional derivatives of L in
    v0, each supported on the same 512 particles, the gradient rows of
    those particles and dL/dB, dL/dalpha agree with the FP64 oracle adjoint
    (itself pinned to central finite differences) within 1e-3."""
    from paper_2009_14514_amd.diff import DiffRollout
    T = torch()
    sc = scenes.diff_scene(counts=(37, 74, 37), box=(2.0, 1.0, 1.0))
    model = DiffRollout(sc, n_sub=16, ckpt_every=4)
    try:
        x0 = T.tensor(sc.pos, dtype=T.float32, device="cuda")
        v0 = T.tensor(sc.vel, dtype=T.float32, device="cuda")
        B, alpha = model.B0, model.alpha0
        xT, _ = model.forward(x0, v0, B, alpha)
        cfg = oracle.cfg_from_params(sc.params)
        x0h = x0.cpu().numpy().astype(np.float64)
        v0h = v0.cpu().numpy().astype(np.float64)
        # target: the GPU's nominal final positions plus the seeded noise
        xhat = xT.cpu().numpy().astype(np.float64) + scenes.target_noise(sc.n, 0.005)
        g = 2.0 * (xT - T.tensor(xhat, dtype=T.float32, device="cuda")) / sc.n
        gx, gv, gB, ga = model.backward(g)
    finally:
        model.close()
    L, rgx, rgv, rgB, rga = oracle.diff_grad(cfg, x0h, v0h, sc.walls, B, alpha, model.dt, 16,
                                             xhat)
    gv = gv.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(11)
    sub = np.sort(rng.choice(sc.n, 512, replace=False))
    assert np.linalg.norm(gv[sub] - rgv[sub]) <= 1e-3 * np.linalg.norm(rgv[sub])
    for _ in range(8):
        d = rng.normal(size=(512, 3))
        dd_gpu = float((gv[sub] * d).sum())
        dd_ref = float((rgv[sub] * d).sum())
        assert abs(dd_gpu - dd_ref) <= 1e-3 * np.linalg.norm(rgv[sub]) * np.linalg.norm(d)
    assert gB == pytest.approx(rgB, rel=1e-3)
    assert ga == pytest.approx(rga, rel=1e-3)


def test_dense_cluster_lists_from_memory():
    # a lattice at 0.7 s: about 190 particles per block, so a block's
    # 27-block neighbourhood (about 5,000 candidates) exceeds the 2,048 LDS
    # slots of the list build; about 780 neighbours per particle
    from paper_2009_14514_amd.diff import DiffRollout
    T = torch()
    base = scenes.diff_scene()
    g = np.arange(0.1, 0.2, 0.007)
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    pos += np.random.default_rng(8).uniform(-1e-4, 1e-4, pos.shape)
    vel = np.zeros_like(pos)
    sc = scenes.Scene("dense", pos, vel, base.walls, dict(base.params))
    model = DiffRollout(sc, n_sub=1, ckpt_every=1, list_cap=1024)
    x0 = T.tensor(pos, dtype=T.float32, device="cuda")
    v0 = T.tensor(vel, dtype=T.float32, device="cuda")
    xT, vT = model.forward(x0, v0, model.B0, model.alpha0)
    model.close()
    cfg = oracle.cfg_from_params(sc.params, nbr_cap=1024)
    x0h = x0.cpu().numpy().astype(np.float64)
    xr, vr = oracle.diff_run(cfg, x0h, vel, sc.walls, model.B0, model.alpha0, model.dt, 1)
    assert np.abs(xT.cpu().numpy() - xr).max() <= 1e-4 * sc.params["spacing"]
    assert np.linalg.norm(vT.cpu().numpy() - vr) <= 1e-4 * np.linalg.norm(vr)


def test_lone_particle_follows_symplectic_euler_in_closed_form():
    """One particle far from the walls: no pair term, so the substeps are
    symplectic Euler under gravity and the adjoint is the identity in x0
    and n dt in v0; the stiffness and viscosity get no gradient."""
    from paper_2009_14514_amd.diff import DiffRollout
    T = torch()
    base = scenes.diff_scene()
    x0n = np.array([[0.15, 0.2, 0.15]])
    v0n = np.array([[0.3, -0.1, 0.2]])
    sc = scenes.Scene("lone", x0n, v0n, base.walls, dict(base.params))
    n = 16
    model = DiffRollout(sc, n_sub=n, ckpt_every=4)
    try:
        x0 = T.tensor(x0n, dtype=T.float32, device="cuda")
        v0 = T.tensor(v0n, dtype=T.float32, device="cuda")
        xT, vT = model.forward(x0, v0, model.B0, model.alpha0)
        dt, g = model.dt, np.asarray(sc.params["gravity"])
        x_cf = x0n + n * dt * v0n + g * dt * dt * n * (n + 1) / 2
        assert np.abs(vT.cpu().numpy() - (v0n + n * dt * g)).max() <= 1e-6
        assert np.abs(xT.cpu().numpy() - x_cf).max() <= 1e-6
        gout = T.full((1, 3), 0.02, dtype=T.float32, device="cuda")
        gx, gv, gB, ga = model.backward(gout)
        assert np.allclose(gx.cpu().numpy(), 0.02, rtol=1e-6, atol=0)
        assert np.allclose(gv.cpu().numpy(), 0.02 * n * dt, rtol=1e-5, atol=0)
        assert gB == 0.0 and ga == 0.0
    finally:
        model.close()
