"""Pins for the oracle's external forces and moving surface: closed-form semi-implicit Euler
under a constant force, an equilibrium that a force balancing gravity must keep, pins that
ignore the force, and translation invariance of a moving surface (cloth and surface shifted
together follow the shifted trajectory, which needs the rebuilt grid, boxes and normals)."""
import numpy as np

import oracle
from paper_2507_11794_amd import workloads as W


def test_free_node_under_constant_external_force_closed_form():
    g = np.array([0.0, -9.81, 0.0])
    m_node, f = 0.002, np.array([0.03, 0.01, -0.02])
    model = oracle.Model(np.array([1.0 / m_node]), np.zeros((0, 2), int), [], [], [], gravity=g)
    model.set_external_force(f.reshape(1, 3))
    x0, v0 = np.array([[0.1, 0.2, 0.3]]), np.array([[0.5, -0.1, 0.0]])
    h, n = 1e-3, 250
    x, v = model.run(x0, v0, h, n)
    a = g + f / m_node
    # v_n = v0 + n h a;  x_n = x0 + sum_{s=1..n} h v_s = x0 + n h v0 + h^2 a n (n + 1) / 2
    assert np.allclose(v, v0 + n * h * a, rtol=0, atol=1e-12)
    assert np.allclose(x, x0 + n * h * v0 + h * h * a * n * (n + 1) / 2, rtol=0, atol=1e-12)
    model.set_external_force(None)
    x2, _ = model.run(x0, v0, h, n)
    assert np.allclose(x2, x0 + n * h * v0 + h * h * g * n * (n + 1) / 2, rtol=0, atol=1e-12)


def test_force_balancing_gravity_keeps_a_relaxed_cloth_at_rest():
    inp = W.config0(n=8)
    flat = W.flat_grid(8, 8, 0.01)
    rest = np.linalg.norm(flat[inp.ends[:, 1]] - flat[inp.ends[:, 0]], axis=1)  # FP64, exact
    w = np.where(inp.pinned.astype(bool), 0.0, 1.0 / inp.mass.astype(np.float64))
    model = oracle.Model(w, inp.ends, rest, inp.k, inp.c, gravity=inp.gravity)
    g = np.asarray(inp.gravity, np.float64)
    f = -np.asarray(inp.mass, np.float64)[:, None] * g[None, :]
    model.set_external_force(f)
    x, v = model.run(flat, np.zeros_like(flat), 1.0 / 2400.0, 200)
    assert np.abs(x - flat).max() < 1e-12 and np.abs(v).max() < 1e-10


def test_pinned_nodes_ignore_external_force():
    inp = W.config0(n=6)
    model = oracle.Model.from_inputs(inp)
    rng = np.random.default_rng(3)
    model.set_external_force(rng.normal(0, 0.05, size=(inp.n_nodes, 3)))
    x, v = model.run(inp.x0, inp.v0, 1.0 / 2400.0, 50)
    pins = inp.pinned.astype(bool)
    assert np.array_equal(x[pins], inp.x0[pins].astype(np.float64)) and not v[pins].any()
    assert np.abs(x[~pins] - inp.x0[~pins]).max() > 1e-4


def _moved_runs(R, d, n_sub=320):
    """The scene as given, and the same scene with cloth, surface and gravity moved by the
    rigid motion p -> R p + d (the surface through set_surface, after construction)."""
    inp = W.small_collision_scene(n=12, freq=4, drop=0.17, spacing=0.02)
    h = 1.0 / 2400.0
    ref = oracle.Model.from_inputs(inp)
    w = np.where(inp.pinned.astype(bool), 0.0, 1.0 / inp.mass.astype(np.float64))
    moved = oracle.Model(w, inp.ends, inp.rest, inp.k, inp.c,
                         gravity=R @ np.asarray(inp.gravity, np.float64), verts=inp.verts,
                         tris=inp.tris, thickness=inp.thickness, restitution=inp.restitution,
                         cell=inp.cell_size)
    moved.set_surface(inp.verts.astype(np.float64) @ R.T + d)
    x0 = inp.x0.astype(np.float64)
    xa, va = x0.copy(), np.zeros_like(x0)
    xb, vb = x0 @ R.T + d, np.zeros_like(x0)
    contacts = 0
    for _ in range(n_sub):
        xa, va, cnt, _m = ref.substep(xa, va, h)
        xb, vb, _c, _m = moved.substep(xb, vb, h)
        contacts += int(np.count_nonzero(cnt))
    return xa, va, xb, vb, contacts


def test_moving_surface_translation_invariance():
    d = np.array([0.37, -0.21, 0.113])
    xa, va, xb, vb, contacts = _moved_runs(np.eye(3), d)
    assert contacts > 1000
    assert np.abs((xb - d) - xa).max() < 1e-9 and np.abs(vb - va).max() < 1e-6


def test_moving_surface_rotation_invariance():
    # a rotation also changes every triangle normal, so a stale normal or box fails here
    q, _ = np.linalg.qr(np.random.default_rng(8).normal(size=(3, 3)))
    R = q if np.linalg.det(q) > 0 else -q
    d = np.array([-0.05, 0.4, 0.2])
    xa, va, xb, vb, contacts = _moved_runs(R, d)
    assert contacts > 1000
    assert np.abs((xb - d) @ R - xa).max() < 1e-9 and np.abs(vb @ R - va).max() < 1e-6


def test_surface_update_takes_effect_between_substeps_only():
    inp = W.small_collision_scene(n=12, freq=4, drop=0.17, spacing=0.02)
    h = 1.0 / 2400.0
    V0 = inp.verts.astype(np.float64)
    V1 = V0 + np.array([0.0, 0.01, 0.0])
    a = oracle.Model.from_inputs(inp)
    x, v = a.run(inp.x0, inp.v0, h, 120)
    a.set_surface(V1)
    x, v = a.run(x, v, h, 60)
    b0 = oracle.Model.from_inputs(inp)
    y, w = b0.run(inp.x0, inp.v0, h, 120)
    b1 = oracle.Model.from_inputs(inp)
    b1.set_surface(V1)
    y, w = b1.run(y, w, h, 60)
    assert np.array_equal(x, y) and np.array_equal(v, w)
    # the lifted surface pushes the resting cloth: the runs differ from a static surface
    c = oracle.Model.from_inputs(inp)
    z, _ = c.run(inp.x0, inp.v0, h, 180)
    assert np.abs(z - x).max() > 1e-4
