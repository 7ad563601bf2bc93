"""Pins for the oracle's time integration: closed forms of the semi-implicit Euler scheme
(single damped spring; free fall) and pinned-node invariants."""
import numpy as np
import pytest

import oracle
from paper_2507_11794_amd import workloads as W


def single_spring_closed_form(e0, v0, k, c, m, h, n):
    """Extension e_n of a spring with one end pinned, advanced by n semi-implicit Euler
    steps: the 2x2 update (e, v) -> ((1 - h^2 w^2) e + h (1 - h g) v, -h w^2 e + (1 - h g) v),
    w^2 = k/m, g = c/m, has det 1 - h g and trace 2 - h^2 w^2 - h g, so
    e_n = rho^n (A cos n theta + B sin n theta) with rho = sqrt(det), cos theta = tr/(2 rho)."""
    w2, g = k / m, c / m
    rho = np.sqrt(1 - h * g)
    cos_t = (2 - h * h * w2 - h * g) / (2 * rho)
    theta = np.arccos(cos_t)
    e1 = (1 - h * h * w2) * e0 + h * (1 - h * g) * v0
    A = e0
    B = (e1 / rho - A * np.cos(theta)) / np.sin(theta)
    return rho ** n * (A * np.cos(n * theta) + B * np.sin(n * theta))


@pytest.mark.parametrize("c", [0.0, 0.05, 0.3])
def test_single_spring_matches_closed_form(c):
    k, m_, L0, h = 500.0, 1e-3, 0.01, 1.0 / 2400
    e0, v0 = 2e-3, 0.15
    w = np.array([0.0, 1.0 / m_])  # node 0 pinned
    mod = oracle.Model(w, [[0, 1]], [L0], [k], [c], gravity=(0.0, 0.0, 0.0))
    x = np.array([[0.0, 0.0, 0.0], [L0 + e0, 0.0, 0.0]])
    v = np.array([[0.0, 0.0, 0.0], [v0, 0.0, 0.0]])
    for n in range(1, 201):
        x, v, _, _ = mod.substep(x, v, h)
        if n in (1, 2, 7, 50, 200):
            want = single_spring_closed_form(e0, v0, k, c, m_, h, n)
            assert abs((x[1, 0] - L0) - want) <= 1e-12 + 1e-9 * abs(e0)
    assert np.all(x[1, 1:] == 0.0) and np.all(x[0] == 0.0)


def test_single_spring_converges_to_harmonic_motion():
    k, m_, L0, A = 500.0, 1e-3, 0.01, 1e-3
    om = np.sqrt(k / m_)
    T = 0.02
    errs = []
    for n_sub in (200, 400, 800):
        h = T / n_sub
        mod = oracle.Model(np.array([0.0, 1.0 / m_]), [[0, 1]], [L0], [k], [0.0],
                           gravity=(0.0, 0.0, 0.0))
        x, v = mod.run(np.array([[0, 0, 0], [L0 + A, 0, 0]], float), np.zeros((2, 3)), h, n_sub)
        errs.append(abs((x[1, 0] - L0) - A * np.cos(om * T)))
    # first-order in h: the error halves when h halves
    assert errs[1] < 0.6 * errs[0] and errs[2] < 0.6 * errs[1]


def test_free_fall_closed_form():
    rng = np.random.default_rng(0)
    N = 10
    x0 = rng.normal(size=(N, 3))
    v0 = rng.normal(size=(N, 3))
    g = np.array([0.1, -9.81, 0.3])
    h = 1.0 / 2400
    # springs at their rest length with zero relative velocity exert no force: use none
    mod = oracle.Model(np.full(N, 1e3), np.zeros((0, 2)), [], [], [], gravity=g)
    x, v = x0.copy(), v0.copy()
    for n in range(1, 101):
        x, v, _, _ = mod.substep(x, v, h)
    n = 100
    want = x0 + n * h * v0 + g * h * h * n * (n + 1) / 2
    assert np.abs(x - want).max() <= 1e-12
    assert np.abs(v - (v0 + n * h * g)).max() <= 1e-12


def test_pinned_nodes_bitwise_still():
    inp = W.config0(n=12)
    mod = oracle.Model.from_inputs(inp)
    x0 = inp.x0.astype(np.float64)
    x, v = mod.run(x0, np.ones_like(x0) * 0.3, inp.h, 40)
    pins = inp.pinned.astype(bool)
    assert np.array_equal(x[pins], x0[pins])
    assert np.all(v[pins] == 0.0)
    assert np.abs(x[~pins] - x0[~pins]).max() > 1e-4


def test_config0_stable_at_quarter_substep():
    inp = W.config0()
    mod = oracle.Model.from_inputs(inp)
    x, v = mod.run(inp.x0, inp.v0, inp.h, inp.n_steps * inp.n_substeps)
    assert np.all(np.isfinite(x))
    # the cloth hangs below its pins and stays about its own size
    assert x[:, 1].min() < -0.1 and np.abs(x).max() < 1.0
