"""Pins for the oracle's adjoint: the reverse-mode substep against an independent
complex-step tangent (dot-product identity), the rollout gradient against central finite
differences and closed forms, and checkpoint-interval invariance."""
import numpy as np
import pytest

import oracle
from paper_2507_11794_amd import workloads as W


def _contact_state(inp, m, n_sub, seed=0):
    x, v = inp.x0.astype(np.float64), inp.v0.astype(np.float64)
    x, v = m.run(x, v, inp.h, n_sub)
    return x, v


@pytest.fixture(scope="module")
def scene():
    inp = W.small_collision_scene(n=14, freq=5, drop=0.165, spacing=0.02)
    m = oracle.Model.from_inputs(inp)
    return inp, m


def test_scene_has_contacts(scene):
    inp, m = scene
    x, v = _contact_state(inp, m, 200)
    _, _, cnt, _ = m.substep(x, v, inp.h)
    assert np.count_nonzero(cnt) >= 5


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_vjp_is_transpose_of_complex_step_tangent(scene, seed):
    inp, m = scene
    x, v = _contact_state(inp, m, 200)
    rng = np.random.default_rng(seed)
    N, S = inp.n_nodes, inp.n_springs
    dx, dv = rng.normal(size=(N, 3)), rng.normal(size=(N, 3))
    dk, dc = rng.normal(size=S) * 50, rng.normal(size=S) * 0.01
    lx, lv = rng.normal(size=(N, 3)), rng.normal(size=(N, 3))
    xr, vr, tx, tv = oracle.substep_jvp_cs(m, x, v, inp.h, dx, dv, dk, dc)
    x1, v1, cnt, _ = m.substep(x, v, inp.h)
    assert np.abs(xr - x1).max() <= 1e-14 and np.abs(vr - v1).max() <= 1e-12
    assert np.count_nonzero(cnt) > 0
    xb, vb, kb, cb = m.substep_vjp(x, v, inp.h, lx, lv)
    lhs = np.sum(tx * lx) + np.sum(tv * lv)
    rhs = np.sum(dx * xb) + np.sum(dv * vb) + np.sum(dk * kb) + np.sum(dc * cb)
    scale = (np.abs(tx * lx).sum() + np.abs(tv * lv).sum())
    assert abs(lhs - rhs) <= 1e-10 * scale


def _loss_and_contacts(m, inp, k, c, v0, n_sub, target):
    m.set_params(k=k, c=c)
    x, v = inp.x0.astype(np.float64), v0.copy()
    sig = []
    for _ in range(n_sub):
        x, v, cnt, _ = m.substep(x, v, inp.h)
        sig.append(cnt.copy())
    return np.mean(np.sum((x - target) ** 2, axis=1)), np.array(sig)


def test_rollout_gradient_vs_central_differences(scene):
    inp, m = scene
    n_sub = 240
    k0, c0 = inp.k.astype(np.float64), inp.c.astype(np.float64)
    v0 = inp.v0.astype(np.float64)
    rng = np.random.default_rng(11)
    k_hat = k0 * (1 + 0.1 * rng.normal(size=k0.shape))
    m.set_params(k=k_hat, c=c0)
    target, _ = m.run(inp.x0, v0, inp.h, n_sub)
    m.set_params(k=k0, c=c0)
    res = m.rollout_grad(inp.x0, v0, inp.h, n_sub, [n_sub], np.zeros((1, inp.n_nodes, 3)), 20)
    xT = res["x_out"][0]
    xbar = (2.0 / inp.n_nodes) * (xT - target)
    g = m.rollout_grad(inp.x0, v0, inp.h, n_sub, [n_sub], xbar[None], 20)
    base, sig0 = _loss_and_contacts(m, inp, k0, c0, v0, n_sub, target)
    checked = 0
    for group, theta, grad, scale in (("k", k0, g["gk"], 300.0), ("c", c0, g["gc"], 0.05),
                                      ("v0", v0, g["gv0"], 0.1)):
        gmax = np.abs(grad).max()
        idx = rng.choice(theta.size, 20, replace=False)
        for i in idx:
            step = 1e-3 * max(abs(theta.flat[i]), scale)
            vals = []
            ok = True
            for sgn in (1, -1):
                th = theta.copy()
                th.flat[i] += sgn * step
                kk, cc, vv = (th, c0, v0) if group == "k" else (k0, th, v0) if group == "c" \
                    else (k0, c0, th)
                L, sig = _loss_and_contacts(m, inp, kk, cc, vv, n_sub, target)
                ok &= np.array_equal(sig, sig0)
                vals.append(L)
            m.set_params(k=k0, c=c0)
            if not ok:
                continue  # a contact flipped inside the FD stencil: the loss is not smooth there
            fd = (vals[0] - vals[1]) / (2 * step)
            assert abs(fd - grad.flat[i]) <= 1e-3 * max(abs(fd), 1e-3 * gmax), (group, i)
            checked += 1
    assert checked >= 40


def test_free_fall_velocity_gradient():
    N, h, n = 5, 1.0 / 2400, 37
    m = oracle.Model(np.full(N, 1e3), np.zeros((0, 2)), [], [], [])
    rng = np.random.default_rng(2)
    xbar = rng.normal(size=(1, N, 3))
    g = m.rollout_grad(rng.normal(size=(N, 3)), rng.normal(size=(N, 3)), h, n, [n], xbar, 7)
    # x_n = x_0 + n h v_0 + (gravity terms)  ->  dL/dv0 = n h xbar, dL/dx0 = xbar
    assert np.allclose(g["gv0"], n * h * xbar[0], rtol=1e-13, atol=0)
    assert np.allclose(g["gx0"], xbar[0], rtol=1e-13, atol=0)


def test_single_spring_stiffness_gradient_matches_closed_form():
    from tests.test_oracle_integrator import single_spring_closed_form
    k, m_, L0, h, c = 500.0, 1e-3, 0.01, 1.0 / 2400, 0.05
    e0, v0, n = 2e-3, 0.15, 90
    mod = oracle.Model(np.array([0.0, 1.0 / m_]), [[0, 1]], [L0], [k], [c], gravity=(0, 0, 0))
    x0 = np.array([[0.0, 0.0, 0.0], [L0 + e0, 0.0, 0.0]])
    v = np.array([[0.0, 0.0, 0.0], [v0, 0.0, 0.0]])
    xbar = np.zeros((1, 2, 3))
    xbar[0, 1, 0] = 1.0  # L = x_1 (n)
    g = mod.rollout_grad(x0, v, h, n, [n], xbar, 9)
    eps = 1e-30  # complex step through the closed form
    dk = single_spring_closed_form(e0, v0, k + 1j * eps, c, m_, h, n).imag / eps
    dc = single_spring_closed_form(e0, v0, k, c + 1j * eps, m_, h, n).imag / eps
    dv0 = single_spring_closed_form(e0, v0 + 1j * eps, k, c, m_, h, n).imag / eps
    assert abs(g["gk"][0] - dk) <= 1e-9 * abs(dk)
    assert abs(g["gc"][0] - dc) <= 1e-9 * abs(dc)
    assert abs(g["gv0"][1, 0] - dv0) <= 1e-9 * abs(dv0)


def test_gradient_independent_of_checkpoint_interval(scene):
    inp, m = scene
    n_sub = 230
    rng = np.random.default_rng(5)
    xbar = rng.normal(size=(2, inp.n_nodes, 3))
    outs = [200, 230]
    ref = m.rollout_grad(inp.x0, inp.v0, inp.h, n_sub, outs, xbar, 1)
    for K in (5, 20, 80, 1000):
        g = m.rollout_grad(inp.x0, inp.v0, inp.h, n_sub, outs, xbar, K)
        for key in ("gk", "gc", "gv0", "gx0", "x_out"):
            assert np.array_equal(g[key], ref[key]), (K, key)
