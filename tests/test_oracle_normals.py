"""Pins for the oracle's per-vertex cloth normals: flat sheets, an exact cylinder, rotation
covariance and the area weighting on a hand-made pair of triangles."""
import numpy as np

import oracle
from paper_2507_11794_amd import workloads as W


def test_flat_cloth_normals_point_up():
    x = W.flat_grid(7, 5, 0.02, (0.3, -1.0, 2.0))
    n = oracle.vertex_normals(7, 5, x)
    assert np.allclose(n, [0.0, 1.0, 0.0], atol=1e-15)


def test_cylinder_interior_normals_are_radial():
    nx, ny, R = 24, 9, 0.7
    th = np.linspace(-1.0, 1.0, nx)
    z = np.linspace(0.0, 0.5, ny)
    x = np.zeros((ny, nx, 3))
    x[..., 0] = R * np.sin(th)[None, :]
    x[..., 1] = R * np.cos(th)[None, :]
    x[..., 2] = z[:, None]
    # j runs along theta (x direction), i along z: with this winding the normals face outward
    n = oracle.vertex_normals(nx, ny, x.reshape(-1, 3)).reshape(ny, nx, 3)
    radial = np.stack([np.sin(th), np.cos(th), np.zeros_like(th)], axis=1)
    inner = n[1:-1, 1:-1]
    assert np.allclose(inner, radial[None, 1:-1], atol=1e-12)


def test_rotation_covariance():
    inp = W.config0(n=9)
    rng = np.random.default_rng(2)
    x = inp.x0.astype(np.float64) + rng.normal(0, 2e-3, size=inp.x0.shape)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    n1 = oracle.vertex_normals(9, 9, x @ q.T)
    n0 = oracle.vertex_normals(9, 9, x)
    assert np.allclose(n1, n0 @ q.T, atol=1e-12)
    assert np.allclose(np.linalg.norm(n0, axis=1), 1.0)


def test_area_weighting_on_a_single_quad():
    # quad a=(0,0,0) b=(0,0,1) c=(1,0,1) d=(1,1,0): triangle (a,b,c) lies in y=0 (normal +y,
    # area 1/2); triangle (a,c,d) has normal (c-a)x(d-a) = (1,0,1)x(1,1,0) = (-1,1,1)
    x = np.array([[0, 0, 0], [1, 1, 0], [0, 0, 1], [1, 0, 1]], dtype=float)  # ids a, d, b, c
    n = oracle.vertex_normals(2, 2, x)
    up, tilt = np.array([0.0, 1.0, 0.0]), np.array([-1.0, 1.0, 1.0])
    for v, want in ((0, up + tilt), (3, up + tilt), (2, up), (1, tilt)):
        assert np.allclose(n[v], want / np.linalg.norm(want), atol=1e-15), v
