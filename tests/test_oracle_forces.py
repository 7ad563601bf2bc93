"""Pins for the oracle's spring forces (Alg. 1): invariants of central pairwise forces,
energy / dissipation-function gradients, and a hand-worked two-node case."""
import numpy as np
import pytest

import oracle
from paper_2507_11794_amd import workloads as W


def _model(inp, **kw):
    return oracle.Model.from_inputs(inp, **kw)


def _state(inp, seed, vscale=0.1, xscale=2e-3):
    rng = np.random.default_rng(seed)
    x = inp.x0.astype(np.float64) + rng.normal(0, xscale, size=inp.x0.shape)
    v = rng.normal(0, vscale, size=inp.x0.shape)
    return x, v


def test_zero_force_at_rest():
    inp = W.config0()
    m = _model(inp)
    flat = W.flat_grid(inp.nx, inp.ny, 0.01)
    # rest lengths of the unjittered grid are rounded to FP32; use the FP64 grid scaled
    # so that each spring is exactly at its stored rest length is not possible, so bound
    # the force by k * (rounding of L0) instead
    F = m.forces(flat, np.zeros_like(flat))
    lw = np.abs(np.linalg.norm(flat[inp.ends[:, 1]] - flat[inp.ends[:, 0]], axis=1)
                - inp.rest.astype(np.float64))
    bound = 12 * 500.0 * lw.max() + 1e-12
    assert np.abs(F).max() <= bound
    # with rest lengths taken from the FP64 grid itself the force vanishes to round-off
    m2 = oracle.Model(np.ones(inp.n_nodes) / 1e-3, inp.ends,
                      np.linalg.norm(flat[inp.ends[:, 1]] - flat[inp.ends[:, 0]], axis=1),
                      inp.k, inp.c)
    assert np.abs(m2.forces(flat, np.zeros_like(flat))).max() <= 1e-12


def test_momentum_and_angular_momentum_conserved():
    inp = W.config0()
    m = _model(inp)
    x, v = _state(inp, 3)
    F = m.forces(x, v)
    scale = np.abs(F).sum()
    assert np.abs(F.sum(axis=0)).max() <= 1e-12 * scale
    torque = np.cross(x, F).sum(axis=0)
    assert np.abs(torque).max() <= 1e-12 * scale * np.abs(x).max()


def test_translation_invariance_and_rotation_covariance():
    inp = W.config0()
    m = _model(inp)
    x, v = _state(inp, 4)
    F = m.forces(x, v)
    Ft = m.forces(x + np.array([3.0, -1.5, 0.25]), v + np.array([0.5, 0.0, -0.2]))
    assert np.abs(F - Ft).max() <= 1e-9 * np.abs(F).max()
    q, _ = np.linalg.qr(np.random.default_rng(8).normal(size=(3, 3)))
    Fr = m.forces(x @ q.T, v @ q.T)
    assert np.abs(Fr - F @ q.T).max() <= 1e-11 * np.abs(F).max()


def test_elastic_force_is_minus_energy_gradient():
    inp = W.config0(n=6)
    m = _model(inp, c=np.zeros(inp.n_springs))
    x, _ = _state(inp, 5)
    zero = np.zeros_like(x)
    a, b = inp.ends[:, 0], inp.ends[:, 1]

    def energy(xx):
        ell = np.linalg.norm(xx[b] - xx[a], axis=1)
        return 0.5 * np.sum(inp.k.astype(np.float64) * (ell - inp.rest.astype(np.float64)) ** 2)

    F = m.forces(x, zero)
    eps = 1e-7
    G = np.zeros_like(x)
    for i in range(x.shape[0]):
        for q in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, q] += eps
            xm[i, q] -= eps
            G[i, q] = (energy(xp) - energy(xm)) / (2 * eps)
    assert np.abs(F + G).max() <= 1e-6 * np.abs(F).max()


def test_damping_force_is_minus_dissipation_gradient_and_dissipates():
    inp = W.config0(n=6)
    m = _model(inp)
    x, v = _state(inp, 6)
    a, b = inp.ends[:, 0], inp.ends[:, 1]
    c = inp.c.astype(np.float64)

    def rayleigh(vv):
        d = x[b] - x[a]
        u = d / np.linalg.norm(d, axis=1, keepdims=True)
        return 0.5 * np.sum(c * np.sum((vv[b] - vv[a]) * u, axis=1) ** 2)

    Fd = m.forces(x, v) - m.forces(x, np.zeros_like(v))
    eps = 1e-6
    G = np.zeros_like(v)
    for i in range(v.shape[0]):
        for q in range(3):
            vp, vm = v.copy(), v.copy()
            vp[i, q] += eps
            vm[i, q] -= eps
            G[i, q] = (rayleigh(vp) - rayleigh(vm)) / (2 * eps)
    assert np.abs(Fd + G).max() <= 1e-7 * np.abs(Fd).max()
    assert np.sum(Fd * v) < 0


def test_two_node_worked_example():
    # Two unit-mass nodes 1.3 m apart on x, rest length 1 m, k = 10 N/m, c = 2 N s/m,
    # node b moving away from a at 0.5 m/s.  Hooke: |f| = 10 * 0.3 = 3 N pulling the nodes
    # together; damping 2 * 0.5 = 1 N opposing the separation: total 4 N toward each other.
    m = oracle.Model(np.ones(2), [[0, 1]], [1.0], [10.0], [2.0])
    x = np.array([[0.0, 0.0, 0.0], [1.3, 0.0, 0.0]])
    v = np.array([[0.0, 0.0, 0.0], [0.5, 0.0, 0.0]])
    F = m.forces(x, v)
    assert np.allclose(F, [[4.0, 0, 0], [-4.0, 0, 0]], atol=1e-12)
    # compressed spring pushes apart; transverse velocity adds no damping force
    x2 = np.array([[0.0, 0.0, 0.0], [0.0, 0.8, 0.0]])
    v2 = np.array([[0.0, 0.0, 0.0], [0.7, 0.0, 0.0]])
    F2 = m.forces(x2, v2)
    assert np.allclose(F2, [[0, -2.0, 0], [0, 2.0, 0]], atol=1e-12)
