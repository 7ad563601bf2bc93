"""Pins for the oracle's collision stage: point-triangle distance against brute force, the
Alg. 2 response on hand-worked flat and creased surfaces, the FP32 broad-phase predicate,
and no penetration of a closed surface over a drop."""
import numpy as np
import pytest

import oracle
from paper_2507_11794_amd import workloads as W


# ---------------------------------------------------------------- point-triangle distance

def _dense_min_dist2(p, A, B, C, n=400):
    s = np.linspace(0.0, 1.0, n + 1)
    u, v = np.meshgrid(s, s, indexing="ij")
    keep = u + v <= 1.0
    u, v = u[keep], v[keep]
    P = A[None] + u[:, None] * (B - A)[None] + v[:, None] * (C - A)[None]
    return np.min(np.sum((P - p[None]) ** 2, axis=1))


def test_point_triangle_distance_vs_dense_sampling():
    rng = np.random.default_rng(0)
    for trial in range(300):
        A, B, C = rng.normal(size=(3, 3))
        if np.linalg.norm(np.cross(B - A, C - A)) < 0.2:
            continue
        p = rng.normal(size=3) * 1.5
        d2 = oracle.point_tri_dist2(p, A, B, C)
        samp = _dense_min_dist2(p, A, B, C)
        # the exact minimum is never above any sample, and the sample grid is fine enough
        # that the true minimum lies within its spacing of the best sample
        assert d2 <= samp + 1e-12
        h = max(np.linalg.norm(B - A), np.linalg.norm(C - A)) / 400
        assert np.sqrt(samp) - np.sqrt(d2) <= 2 * h + 1e-12


def test_point_triangle_distance_regions():
    A, B, C = np.array([0.0, 0, 0]), np.array([1.0, 0, 0]), np.array([0.0, 1, 0])
    # above the interior: plane distance
    assert np.isclose(oracle.point_tri_dist2([0.2, 0.2, 0.7], A, B, C), 0.49)
    # beside vertex B
    assert np.isclose(oracle.point_tri_dist2([2.0, -1.0, 0.0], A, B, C), 2.0)
    # beside the hypotenuse
    assert np.isclose(oracle.point_tri_dist2([1.0, 1.0, 0.0], A, B, C), 0.5)


# ---------------------------------------------------------------- response, worked examples

def _single_node_model(verts, tris, th=0.005, r=0.5):
    return oracle.Model(np.array([1e3]), np.zeros((0, 2)), [], [], [], gravity=(0, 0, 0),
                        verts=verts, tris=tris, thickness=th, restitution=r, cell=0.05)


def _square(y=0.0):
    verts = np.array([[0, y, 0], [1, y, 0], [1, y, 1], [0, y, 1]], dtype=np.float64)
    tris = np.array([[0, 2, 1], [0, 3, 2]])  # normals +y
    return verts, tris


def test_flat_plane_push_to_thickness_and_halved_reversed_velocity():
    verts, tris = _square()
    m = _single_node_model(verts, tris)
    A, n, _, _ = m.triangle(0)
    assert np.allclose(n, [0, 1, 0])
    h = 1.0 / 2400
    x = np.array([[0.3, 0.004, 0.6]])
    v = np.array([[0.8, -2.0, 0.1]])
    x1, v1, cnt, _ = m.substep(x, v, h)
    xs = x + h * v  # no forces, no gravity
    assert cnt[0] == 1
    assert abs(x1[0, 1] - 0.005) <= 1e-15
    assert np.allclose(x1[0, [0, 2]], xs[0, [0, 2]], atol=0, rtol=1e-15)
    assert np.array_equal(v1, -0.5 * v)


def test_flat_plane_two_hits_average_equals_single_push():
    verts, tris = _square()
    m = _single_node_model(verts, tris)
    x = np.array([[0.5, -0.001, 0.5]])  # on the shared diagonal, below the plane
    x1, v1, cnt, _ = m.substep(x, np.zeros((1, 3)), 1.0 / 2400)
    assert cnt[0] == 2
    assert abs(x1[0, 1] - 0.005) <= 1e-15


def test_crease_average_of_two_pushes():
    # two triangles meeting at the x axis: one in the y=0 plane (normal +y), one in the
    # x-y plane (normal -z) -- a node near the crease gets the mean of the two pushes
    verts = np.array([[0, 0, 0], [1, 0, 0], [0, 0, 1], [0, 1, 0]], dtype=np.float64)
    tris = np.array([[0, 2, 1], [0, 3, 1]])
    m = _single_node_model(verts, tris, th=0.01)
    _, n0, _, _ = m.triangle(0)
    _, n1, _, _ = m.triangle(1)
    assert np.allclose(n0, [0, 1, 0]) and np.allclose(n1, [0, 0, -1])
    p = np.array([0.4, 0.002, -0.003])
    x1, _, cnt, _ = m.substep(p[None], np.zeros((1, 3)), 1e-9)
    assert cnt[0] == 2
    want = p + 0.5 * ((0.01 - 0.002) * n0 + (0.01 - 0.003) * n1)
    assert np.allclose(x1[0], want, atol=1e-15)


def test_strict_threshold_and_pins_never_collide():
    verts, tris = _square()
    m = _single_node_model(verts, tris, th=0.25)  # 0.25 and 0.5 are exact binary values
    x1, _, cnt, _ = m.substep(np.array([[0.5, 0.25, 0.25]]), np.zeros((1, 3)), 1e-12)
    assert cnt[0] == 0 and x1[0, 1] == 0.25
    pinned = oracle.Model(np.array([0.0]), np.zeros((0, 2)), [], [], [], verts=verts, tris=tris,
                          thickness=0.25)
    x2, v2, cnt2, _ = pinned.substep(np.array([[0.5, 0.01, 0.5]]), np.ones((1, 3)), 0.1)
    assert cnt2[0] == 0 and x2[0, 1] == 0.01 and np.all(v2 == 0)


# ---------------------------------------------------------------- candidate sets

def test_bucket_grid_never_changes_contacts():
    inp = W.small_collision_scene()
    m = oracle.Model.from_inputs(inp)
    rng = np.random.default_rng(3)
    V = inp.verts.astype(np.float64)
    P = V[rng.integers(0, V.shape[0], 400)] + rng.normal(0, 0.006, size=(400, 3))
    for p in P:
        got = m.contacts(p)
        brute = [t for t in range(inp.n_tris)
                 if oracle.point_tri_dist2(p, *V[inp.tris[t]]) < inp.thickness ** 2]
        assert list(got) == brute


def test_fp32_candidates_contain_every_contact_and_respect_box_faces():
    inp = W.small_collision_scene()
    V = inp.verts
    rng = np.random.default_rng(4)
    P = (V[rng.integers(0, V.shape[0], 300)].astype(np.float64)
         + rng.normal(0, 0.006, size=(300, 3))).astype(np.float32)
    pairs = oracle.candidates_f32(P, V, inp.tris, inp.thickness)
    cand = set(map(tuple, pairs))
    V64 = V.astype(np.float64)
    for i, p in enumerate(P.astype(np.float64)):
        for t in range(inp.n_tris):
            if oracle.point_tri_dist2(p, *V64[inp.tris[t]]) < inp.thickness ** 2:
                assert (i, t) in cand
    # ordering: ascending node, then triangle
    key = pairs[:, 0].astype(np.int64) * inp.n_tris + pairs[:, 1]
    assert np.all(np.diff(key) > 0)
    # inclusive box: a point exactly on the inflated box corner is in, one ulp out is not
    th = np.float32(0.005)
    tri = np.array([[0, 1, 2]])
    verts = np.array([[0.1, 0.2, 0.3], [0.4, 0.25, 0.35], [0.2, 0.6, 0.31]], dtype=np.float32)
    lo = verts.min(axis=0) - th
    hi = verts.max(axis=0) + th
    on = np.stack([lo, hi]).astype(np.float32)
    assert oracle.candidates_f32(on, verts, tri, th).shape[0] == 2
    out = np.stack([np.nextafter(lo, np.float32(-1)), np.nextafter(hi, np.float32(2))])
    assert oracle.candidates_f32(out.astype(np.float32), verts, tri, th).shape[0] == 0


# ---------------------------------------------------------------- whole step, no penetration

def _inside_closed_mesh(P, V, F):
    """Crossing-number test along +x with a ray-triangle intersection per triangle."""
    A, B, C = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    e1, e2 = B - A, C - A
    d = np.array([1.0, 0.0, 0.0]) + np.array([0.0, 1e-7, 3e-7])  # avoid grazing edges
    inside = np.zeros(P.shape[0], dtype=bool)
    hvec = np.cross(d[None], e2)
    a = np.einsum("ij,ij->i", e1, hvec)
    for k, p in enumerate(P):
        s = p[None] - A
        f = 1.0 / a
        u = f * np.einsum("ij,ij->i", s, hvec)
        q = np.cross(s, e1)
        v = f * (q @ d)
        t = f * np.einsum("ij,ij->i", e2, q)
        hit = (np.abs(a) > 1e-14) & (u >= 0) & (v >= 0) & (u + v <= 1) & (t > 0)
        inside[k] = np.count_nonzero(hit) % 2 == 1
    return inside


def test_drop_never_penetrates_surface():
    inp = W.small_collision_scene(n=20, n_steps=120)
    m = oracle.Model.from_inputs(inp)
    V = inp.verts.astype(np.float64)
    x, v = inp.x0.astype(np.float64), inp.v0.astype(np.float64)
    touched = 0
    for s in range(inp.n_steps * inp.n_substeps):
        x, v, cnt, _ = m.substep(x, v, inp.h)
        touched = max(touched, int(np.count_nonzero(cnt)))
        if s % 8 == 7:
            assert not np.any(_inside_closed_mesh(x, V, inp.tris))
    assert touched > 20  # the drop really reached the surface


def test_fast_inside_test_equals_the_ray_parity_brute_force():
    """oracle.inside (segment crossings from the centre, candidate triangles from a k-d tree
    of directions) against the brute-force ray parity along +x over every triangle, on points
    around a displaced sphere: near its surface, deep inside, far outside."""
    from oracle.inside import inside_closed_mesh

    verts, tris = W.displaced_sphere(6, 0.15, 0.015, np.random.default_rng(8))
    V = verts.astype(np.float64)
    rng = np.random.default_rng(9)
    P = np.concatenate([
        V[rng.integers(0, V.shape[0], 600)] * (1 + rng.normal(0, 0.02, size=(600, 1))),
        rng.normal(0, 0.05, size=(100, 3)),
        rng.uniform(-0.4, 0.4, size=(300, 3)),
    ])
    fast = inside_closed_mesh(P, V, tris)
    slow = _inside_closed_mesh(P, V, tris)
    assert np.array_equal(fast, slow)
    assert 100 < fast.sum() < P.shape[0] - 100
