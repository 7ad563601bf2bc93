"""Seeded input generators: counts, topology and orientation fixed by closed forms."""
import numpy as np
import pytest

from paper_2507_11794_amd import workloads as W


@pytest.mark.parametrize("nx,ny", [(2, 2), (3, 5), (32, 32), (17, 4), (316, 316)])
def test_spring_count_closed_form(nx, ny):
    ends, kind = W.grid_topology(nx, ny)
    assert ends.shape[0] == W.spring_count(nx, ny)
    if nx == ny:
        n = nx
        assert ends.shape[0] == 6 * n * n - 10 * n + 2
    # no self springs, no duplicates
    assert np.all(ends[:, 0] != ends[:, 1])
    key = np.sort(ends, axis=1)
    assert np.unique(key, axis=0).shape[0] == ends.shape[0]


def test_rest_lengths_by_kind():
    inp = W.config0()
    s = 0.01
    want = np.array([s, s * np.sqrt(2.0), 2 * s], dtype=np.float64)[inp.kind]
    assert np.array_equal(inp.rest, want.astype(np.float32))


@pytest.mark.parametrize("m", [1, 2, 3, 6, 10, 16])
def test_geodesic_sphere_counts_and_closure(m):
    P, F = W.geodesic_sphere(m)
    assert P.shape[0] == 10 * m * m + 2
    assert F.shape[0] == 20 * m * m
    e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]])
    # closed 2-manifold: each undirected edge is used exactly twice, once per direction
    und = np.sort(e, axis=1)
    _, cnt = np.unique(und, axis=0, return_counts=True)
    assert np.all(cnt == 2)
    V, E = P.shape[0], und.shape[0] // 2
    assert V - E + F.shape[0] == 2
    assert np.allclose(np.linalg.norm(P, axis=1), 1.0)


def test_displaced_sphere_orientation_and_amplitude():
    rng = np.random.default_rng(5)
    V, F = W.displaced_sphere(8, 0.25, 0.02, rng)
    V64 = V.astype(np.float64)
    r = np.linalg.norm(V64, axis=1)
    assert r.max() <= 0.25 + 0.02 + 1e-6 and r.min() >= 0.25 - 0.02 - 1e-6
    assert abs(np.max(np.abs(r - 0.25)) - 0.02) < 1e-6
    a, b, c = V64[F[:, 0]], V64[F[:, 1]], V64[F[:, 2]]
    n = np.cross(b - a, c - a)
    assert np.all(np.einsum("ij,ij->i", n, (a + b + c) / 3) > 0)
    # consistently outward: positive enclosed volume
    vol = np.sum(np.einsum("ij,ij->i", a, np.cross(b, c))) / 6.0
    assert vol > 0
    # directed edges appear once each (consistent winding)
    e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]])
    assert np.unique(e, axis=0).shape[0] == e.shape[0]


def test_noise_vanishes_on_lattice_points():
    perm = W.improved_noise_perm(np.random.default_rng(0))
    P = np.random.default_rng(1).integers(-20, 20, size=(200, 3)).astype(np.float64)
    assert np.all(W.improved_noise(P, perm) == 0.0)
    Q = np.random.default_rng(2).uniform(-10, 10, size=(5000, 3))
    val = W.improved_noise(Q, perm)
    assert np.all(np.abs(val) <= 1.5) and np.std(val) > 0.05


def test_seeds_reproduce_bitwise():
    a, b = W.config1(n=40, freq=8), W.config1(n=40, freq=8)
    for f in ("x0", "verts", "tris", "ends", "rest", "k", "c"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
    c = W.config1(n=40, freq=8, seed=99)
    assert not np.array_equal(a.x0, c.x0)


def test_config_shapes():
    c0 = W.config0()
    assert (c0.n_nodes, c0.n_springs, int(c0.pinned.sum())) == (1024, 5826, 2)
    assert c0.pinned[0] == 1 and c0.pinned[31] == 1
    jit = c0.x0.astype(np.float64) - W.flat_grid(32, 32, 0.01)
    assert 5e-5 < np.std(jit) < 2e-4
    c4, k_hat = W.config4()
    assert c4.n_nodes == 4096 and c4.n_springs == 23938 and c4.n_tris == 2000
    rel = k_hat.astype(np.float64) / c4.k - 1.0
    assert 0.05 < np.std(rel) < 0.15
    batch = W.config3(n_cloths=6)
    for b in batch:
        assert 16 <= b.nx <= 128 and b.n_tris == 5120
        ks = b.k[b.kind == W.STRUCT][0]
        assert 100.0 <= ks <= 2000.0
        assert np.allclose(b.k[b.kind == W.SHEAR], 0.4 * ks, rtol=1e-6)
