"""Seeded synthetic inputs for the mass-spring cloth step.

This module builds input arrays only: cloth grids, spring lists, surface meshes and the
scene parameters that go with them.  It holds none of the simulation's arithmetic (no
forces, integration, broad phase or collision), so both the HIP path and the FP64 oracle
can consume what it produces without sharing any code of the method.

Scene shapes follow the paper's workloads: a square mass-spring cloth (Sec. 3, Alg. 1)
hanging from pinned corners (Sec. 4.1, the hanging-cloth scene) or dropped onto a static
surface of up to 100K triangles (Sec. 4.2, whose Dragon model has 50K vertices / 100K
triangles).  The paper's scanned meshes are not available, so a seeded, radially
displaced geodesic icosphere of matching size stands in for them; frequency m gives
20 m^2 triangles and 10 m^2 + 2 vertices (m = 71 gives 100,820 / 50,412).

All arrays are FP32 (positions, masses, spring parameters) or int32 (indices), the
precision the C ABI takes.  Random draws use numpy's PCG64 ``default_rng`` in FP64 and
are cast once to FP32.
"""
from __future__ import annotations

import dataclasses
import functools
import math
from typing import List, Optional

import numpy as np

# Spring kinds (structural / shear / bend), the usual mass-spring cloth topology.
STRUCT, SHEAR, BEND = 0, 1, 2

GRAVITY = (0.0, -9.81, 0.0)


@dataclasses.dataclass
class ClothInputs:
    """One cloth scene: everything cloth_create takes, plus the stepping schedule."""

    nx: int
    ny: int
    x0: np.ndarray          # [N,3] float32, AoS
    v0: np.ndarray          # [N,3] float32
    mass: np.ndarray        # [N] float32
    pinned: np.ndarray      # [N] uint8
    ends: np.ndarray        # [S,2] int32
    rest: np.ndarray        # [S] float32
    k: np.ndarray           # [S] float32
    c: np.ndarray           # [S] float32
    kind: np.ndarray        # [S] int8 (STRUCT/SHEAR/BEND); informational
    verts: np.ndarray       # [V,3] float32 (may be empty)
    tris: np.ndarray        # [T,3] int32, CCW seen from outside (may be empty)
    gravity: tuple = GRAVITY
    thickness: float = 0.0  # m; 0 disables collision
    cell_size: float = 0.0  # m; grid cell edge for the broad phase
    restitution: float = 0.5
    dt: float = 1.0 / 600.0
    n_substeps: int = 4
    n_steps: int = 100
    name: str = ""

    @property
    def n_nodes(self) -> int:
        return self.nx * self.ny

    @property
    def n_springs(self) -> int:
        return int(self.ends.shape[0])

    @property
    def n_tris(self) -> int:
        return int(self.tris.shape[0])

    @property
    def h(self) -> float:
        return self.dt / self.n_substeps


# ----------------------------------------------------------------------------- cloth


def spring_count(nx: int, ny: int) -> int:
    """Number of structural + shear + bend springs of an nx-by-ny grid."""
    struct = ny * (nx - 1) + nx * (ny - 1)
    shear = 2 * (nx - 1) * (ny - 1)
    bend = ny * max(nx - 2, 0) + nx * max(ny - 2, 0)
    return struct + shear + bend


def grid_topology(nx: int, ny: int):
    """Springs of an nx-by-ny node grid, node (i, j) = row i, column j, id i*nx + j.

    Structural springs join 4-neighbours, shear springs both diagonals of each quad and
    bend springs nodes two apart along a row or column.  Returns ``ends`` [S,2] int32 and
    ``kind`` [S] int8.
    """
    ids = np.arange(nx * ny, dtype=np.int64).reshape(ny, nx)
    parts, kinds = [], []

    def add(a, b, kd):
        a = a.ravel()
        b = b.ravel()
        parts.append(np.stack([a, b], axis=1))
        kinds.append(np.full(a.shape[0], kd, dtype=np.int8))

    add(ids[:, :-1], ids[:, 1:], STRUCT)          # (i,j)-(i,j+1)
    add(ids[:-1, :], ids[1:, :], STRUCT)          # (i,j)-(i+1,j)
    add(ids[:-1, :-1], ids[1:, 1:], SHEAR)        # (i,j)-(i+1,j+1)
    add(ids[:-1, 1:], ids[1:, :-1], SHEAR)        # (i,j+1)-(i+1,j)
    if nx > 2:
        add(ids[:, :-2], ids[:, 2:], BEND)        # (i,j)-(i,j+2)
    if ny > 2:
        add(ids[:-2, :], ids[2:, :], BEND)        # (i,j)-(i+2,j)
    ends = np.concatenate(parts).astype(np.int32)
    kind = np.concatenate(kinds)
    return ends, kind


def flat_grid(nx: int, ny: int, spacing: float, origin=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Unjittered node positions [N,3] float64 in the x-z plane: node (i,j) at
    origin + (j*s, 0, i*s)."""
    i, j = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64),
                       indexing="ij")
    p = np.zeros((ny, nx, 3), dtype=np.float64)
    p[..., 0] = origin[0] + j * spacing
    p[..., 1] = origin[1]
    p[..., 2] = origin[2] + i * spacing
    return p.reshape(-1, 3)


def make_cloth(nx: int, ny: int, spacing: float, origin, k_struct: float, k_shear: float,
               k_bend: float, damping: float, mass: float, pins, rng: np.random.Generator,
               jitter: float = 1e-4):
    """A flat cloth with seeded N(0, jitter) position noise on all coordinates.

    Rest lengths come from the unjittered grid.  ``pins`` lists (row, col) pairs.
    """
    flat = flat_grid(nx, ny, spacing, origin)
    ends, kind = grid_topology(nx, ny)
    rest64 = np.linalg.norm(flat[ends[:, 1]] - flat[ends[:, 0]], axis=1)
    kval = np.array([k_struct, k_shear, k_bend], dtype=np.float64)[kind]
    x0 = (flat + rng.normal(0.0, jitter, size=flat.shape)).astype(np.float32)
    pinned = np.zeros(nx * ny, dtype=np.uint8)
    for (r, cidx) in pins:
        pinned[r * nx + cidx] = 1
    return dict(
        nx=nx, ny=ny, x0=x0,
        v0=np.zeros((nx * ny, 3), dtype=np.float32),
        mass=np.full(nx * ny, mass, dtype=np.float32),
        pinned=pinned, ends=ends,
        rest=rest64.astype(np.float32),
        k=kval.astype(np.float32),
        c=np.full(ends.shape[0], damping, dtype=np.float32),
        kind=kind,
    )


# --------------------------------------------------------------------------- surface


def _icosahedron():
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]],
                 dtype=np.int64)
    return v, f


def geodesic_sphere(freq: int):
    P, F = _geodesic_sphere_cached(int(freq))
    return P.copy(), F.copy()


@functools.lru_cache(maxsize=8)
def _geodesic_sphere_cached(freq: int):
    """Class-I geodesic subdivision of the icosahedron at frequency ``freq``.

    Each face (A, B, C) is cut into freq^2 triangles on the lattice
    P(a, b) = ((freq-a-b) A + a B + b C) / freq; lattice points shared by faces are merged
    through an exact integer key.  Returns unit vectors [V,3] float64 and triangles [T,3]
    int64 with V = 10 freq^2 + 2, T = 20 freq^2.
    """
    m = int(freq)
    if m < 1:
        raise ValueError("freq must be >= 1")
    base_v, base_f = _icosahedron()
    keys = {}
    pts = []

    def vid(ia, wa, ib, wb, ic, wc):
        items = sorted(((ia, wa), (ib, wb), (ic, wc)))
        key = tuple((i, w) for (i, w) in items if w != 0)
        # merge equal vertex ids (cannot happen for distinct face corners)
        idx = keys.get(key)
        if idx is None:
            idx = len(pts)
            keys[key] = idx
            p = (wa * base_v[ia] + wb * base_v[ib] + wc * base_v[ic]) / m
            pts.append(p)
        return idx

    tris = []
    for (A, B, C) in base_f:
        lat = {}
        for a in range(m + 1):
            for b in range(m + 1 - a):
                lat[(a, b)] = vid(A, m - a - b, B, a, C, b)
        for a in range(m):
            for b in range(m - a):
                tris.append((lat[(a, b)], lat[(a + 1, b)], lat[(a, b + 1)]))
                if a + b + 1 < m:
                    tris.append((lat[(a + 1, b)], lat[(a + 1, b + 1)], lat[(a, b + 1)]))
    P = np.asarray(pts, dtype=np.float64)
    P /= np.linalg.norm(P, axis=1, keepdims=True)
    return P, np.asarray(tris, dtype=np.int64)


def improved_noise_perm(rng: np.random.Generator) -> np.ndarray:
    """A seeded permutation of 0..255, doubled to 512 entries (Perlin 2002)."""
    p = rng.permutation(256).astype(np.int64)
    return np.concatenate([p, p])


def improved_noise(P: np.ndarray, perm: np.ndarray) -> np.ndarray:
    """Perlin's 2002 "improved noise" at points P [n,3] (vectorised numpy).

    Lattice cell from floor, quintic fade 6t^5 - 15t^4 + 10t^3, hashed corner gradients
    taken from the 12 cube-edge directions, trilinear blend.  Values lie in about [-1, 1].
    """
    P = np.asarray(P, dtype=np.float64)
    fl = np.floor(P)
    cell = fl.astype(np.int64) & 255
    f = P - fl
    fade = f * f * f * (f * (f * 6.0 - 15.0) + 10.0)
    X, Y, Z = cell[:, 0], cell[:, 1], cell[:, 2]
    x, y, z = f[:, 0], f[:, 1], f[:, 2]
    u, v, w = fade[:, 0], fade[:, 1], fade[:, 2]

    def grad(hsh, gx, gy, gz):
        hh = hsh & 15
        a = np.where(hh < 8, gx, gy)
        b = np.where(hh < 4, gy, np.where((hh == 12) | (hh == 14), gx, gz))
        return np.where(hh & 1, -a, a) + np.where(hh & 2, -b, b)

    A = perm[X] + Y
    AA = perm[A] + Z
    AB = perm[A + 1] + Z
    B = perm[X + 1] + Y
    BA = perm[B] + Z
    BB = perm[B + 1] + Z

    def lerp(t, a, b):
        return a + t * (b - a)

    x1 = lerp(u, grad(perm[AA], x, y, z), grad(perm[BA], x - 1, y, z))
    x2 = lerp(u, grad(perm[AB], x, y - 1, z), grad(perm[BB], x - 1, y - 1, z))
    y1 = lerp(v, x1, x2)
    x3 = lerp(u, grad(perm[AA + 1], x, y, z - 1), grad(perm[BA + 1], x - 1, y, z - 1))
    x4 = lerp(u, grad(perm[AB + 1], x, y - 1, z - 1), grad(perm[BB + 1], x - 1, y - 1, z - 1))
    y2 = lerp(v, x3, x4)
    return lerp(w, y1, y2)


def displaced_sphere(freq: int, radius: float, amplitude: float, rng: np.random.Generator,
                     center=(0.0, 0.0, 0.0), octaves: int = 3, frequency: float = 4.0):
    """Geodesic sphere with seeded radial gradient-noise displacement.

    r(u) = radius + amplitude * n(u) / max|n|, with n(u) = sum_o 0.5^o * noise(2^o * f * u)
    over ``octaves`` octaves.  Triangles are wound counter-clockwise seen from outside.
    Returns verts [V,3] float32 and tris [T,3] int32.
    """
    U, F = geodesic_sphere(freq)
    perm = improved_noise_perm(rng)
    n = np.zeros(U.shape[0], dtype=np.float64)
    for o in range(octaves):
        n += (0.5 ** o) * improved_noise((2.0 ** o) * frequency * U + 0.5, perm)
    peak = np.max(np.abs(n))
    if amplitude > 0 and peak > 0:
        n *= 1.0 / peak
    r = radius + amplitude * n
    V = (np.asarray(center, dtype=np.float64)[None, :] + r[:, None] * U)
    # orient counter-clockwise seen from outside: normal . (centroid - center) > 0
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    nrm = np.cross(b - a, c - a)
    cen = (a + b + c) / 3.0 - np.asarray(center, dtype=np.float64)[None, :]
    flip = np.einsum("ij,ij->i", nrm, cen) < 0
    F = F.copy()
    F[flip] = F[flip][:, [0, 2, 1]]
    return V.astype(np.float32), F.astype(np.int32)


def mean_edge_length(verts: np.ndarray, tris: np.ndarray) -> float:
    """Mean length of the unique edges of a triangle mesh (FP64 over the FP32 mesh)."""
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]]).astype(np.int64)
    e.sort(axis=1)
    e = np.unique(e, axis=0)
    V = verts.astype(np.float64)
    return float(np.mean(np.linalg.norm(V[e[:, 1]] - V[e[:, 0]], axis=1)))


# --------------------------------------------------------------------------- configs

K_STRUCT, K_SHEAR, K_BEND = 500.0, 200.0, 50.0
DAMPING = 0.05
NODE_MASS = 1e-3


def _inputs(cloth: dict, verts=None, tris=None, **kw) -> ClothInputs:
    if verts is None:
        verts = np.zeros((0, 3), dtype=np.float32)
        tris = np.zeros((0, 3), dtype=np.int32)
    return ClothInputs(verts=verts, tris=tris, **cloth, **kw)


def _surface_cell(verts, tris) -> float:
    return float(np.float32(2.0 * mean_edge_length(verts, tris)))


def config0(seed: int = 1000, n: int = 32, n_steps: int = 100) -> ClothInputs:
    """Hanging cloth, no collision: 32x32, spacing 0.01 m, two corners of row 0 pinned."""
    rng = np.random.default_rng(seed)
    cloth = make_cloth(n, n, 0.01, (0.0, 0.0, 0.0), K_STRUCT, K_SHEAR, K_BEND, DAMPING,
                       NODE_MASS, pins=[(0, 0), (0, n - 1)], rng=rng)
    return _inputs(cloth, dt=1.0 / 600.0, n_substeps=4, n_steps=n_steps,
                   name=f"hanging cloth {n}x{n}")


def config1(seed: int = 1001, surface_seed: int = 2001, n: int = 316, freq: int = 71,
            spacing: Optional[float] = None, n_steps: int = 300) -> ClothInputs:
    """A 1 m square cloth of n x n nodes dropped from y = 0.3 m onto a displaced sphere
    (R = 0.25 m, amplitude 0.02 m) of 20 freq^2 triangles; thickness 5 mm, grid cell
    = the mean surface edge (the thickness is about the edge length here, so a finer grid
    than the usual 2 x mean edge halves the references a node near the surface scans; the
    contacts do not depend on the cell size)."""
    if spacing is None:
        spacing = 1.0 / (n - 1)
    half = 0.5 * spacing * (n - 1)
    rng = np.random.default_rng(seed)
    cloth = make_cloth(n, n, spacing, (-half, 0.3, -half), K_STRUCT, K_SHEAR, K_BEND,
                       DAMPING, NODE_MASS, pins=[], rng=rng)
    verts, tris = displaced_sphere(freq, 0.25, 0.02, np.random.default_rng(surface_seed))
    return _inputs(cloth, verts, tris, thickness=0.005,
                   cell_size=float(np.float32(mean_edge_length(verts, tris))),
                   dt=1.0 / 600.0, n_substeps=4, n_steps=n_steps,
                   name=f"cloth {n}x{n} vs sphere {tris.shape[0]} tris")


def config2(seed: int = 1002, n: int = 800, n_steps: int = 500) -> ClothInputs:
    """High-resolution hanging cloth, 800x800, 4 corners pinned, no collision."""
    rng = np.random.default_rng(seed)
    cloth = make_cloth(n, n, 0.01, (0.0, 0.0, 0.0), K_STRUCT, K_SHEAR, K_BEND, DAMPING,
                       NODE_MASS, pins=[(0, 0), (0, n - 1), (n - 1, 0), (n - 1, n - 1)],
                       rng=rng)
    return _inputs(cloth, dt=1.0 / 1200.0, n_substeps=2, n_steps=n_steps,
                   name=f"hanging cloth {n}x{n}")


def config3(n_cloths: int = 512, seed: int = 3000, side_lo: int = 16, side_hi: int = 128,
            freq: int = 16, n_steps: int = 200) -> List[ClothInputs]:
    """Many independent cloths of uneven sizes, each over its own displaced sphere.

    Side lengths ~ U{side_lo..side_hi}; structural stiffness log-uniform in [100, 2000] N/m
    with shear and bend at 0.4x and 0.1x of it; sphere R = 0.2 m, amplitude 0.02 m."""
    out = []
    for i, ss in enumerate(np.random.SeedSequence(seed).spawn(n_cloths)):
        rng = np.random.default_rng(ss)
        side = int(rng.integers(side_lo, side_hi + 1))
        ks = float(np.exp(rng.uniform(math.log(100.0), math.log(2000.0))))
        half = 0.5 * 0.01 * (side - 1)
        cloth = make_cloth(side, side, 0.01, (-half, 0.3, -half), ks, 0.4 * ks, 0.1 * ks,
                           DAMPING, NODE_MASS, pins=[], rng=rng)
        verts, tris = displaced_sphere(freq, 0.2, 0.02, rng)
        out.append(_inputs(cloth, verts, tris, thickness=0.005,
                           cell_size=_surface_cell(verts, tris), dt=1.0 / 600.0,
                           n_substeps=4, n_steps=n_steps, name=f"batch cloth {i} {side}x{side}"))
    return out


def config4(seed: int = 1004, target_seed: int = 4004, n: int = 64, freq: int = 10,
            n_steps: int = 200):
    """Differentiable scene: 64x64 cloth over a 2,000-triangle displaced sphere, plus a
    target stiffness k_hat = k (1 + 0.1 xi), xi ~ N(0, 1).  Returns (inputs, k_hat)."""
    rng = np.random.default_rng(seed)
    half = 0.5 * 0.01 * (n - 1)
    cloth = make_cloth(n, n, 0.01, (-half, 0.3, -half), K_STRUCT, K_SHEAR, K_BEND, DAMPING,
                       NODE_MASS, pins=[], rng=rng)
    verts, tris = displaced_sphere(freq, 0.2, 0.02, np.random.default_rng(seed + 1))
    inp = _inputs(cloth, verts, tris, thickness=0.005, cell_size=_surface_cell(verts, tris),
                  dt=1.0 / 600.0, n_substeps=4, n_steps=n_steps,
                  name=f"differentiable cloth {n}x{n}")
    xi = np.random.default_rng(target_seed).normal(0.0, 1.0, size=inp.n_springs)
    k_hat = (inp.k.astype(np.float64) * (1.0 + 0.1 * xi)).astype(np.float32)
    return inp, k_hat


def small_collision_scene(n: int = 24, freq: int = 6, seed: int = 7, drop: float = 0.22,
                          spacing: float = 0.015, radius: float = 0.15,
                          n_steps: int = 40) -> ClothInputs:
    """A small cloth-over-sphere scene for tests (a few hundred nodes and triangles)."""
    rng = np.random.default_rng(seed)
    half = 0.5 * spacing * (n - 1)
    cloth = make_cloth(n, n, spacing, (-half, drop, -half), K_STRUCT, K_SHEAR, K_BEND,
                       DAMPING, NODE_MASS, pins=[], rng=rng)
    verts, tris = displaced_sphere(freq, radius, 0.015, np.random.default_rng(seed + 100))
    return _inputs(cloth, verts, tris, thickness=0.005, cell_size=_surface_cell(verts, tris),
                   dt=1.0 / 600.0, n_substeps=4, n_steps=n_steps,
                   name=f"small cloth {n}x{n} vs sphere {tris.shape[0]} tris")


def pulled_cloth_scene(n: int = 24, freq: int = 6, seed: int = 9, spacing: float = 0.015,
                       drop: float = 0.165, pull: float = 0.004, n_steps: int = 120):
    """A cloth dropped onto a sphere whose last row is pulled along +x (the pulled-cloth
    scenes of Sec. 4): returns (inputs, f_ext [N,3] float32 in newtons)."""
    inp = small_collision_scene(n=n, freq=freq, seed=seed, drop=drop, spacing=spacing,
                                n_steps=n_steps)
    f = np.zeros((inp.n_nodes, 3), dtype=np.float32)
    f[(n - 1) * n:, 0] = pull
    inp.name = f"pulled cloth {n}x{n} vs sphere {inp.n_tris} tris"
    return inp, f


def moving_surface(verts: np.ndarray, frame: int, dt: float, velocity=(0.0, 0.04, 0.0),
                   omega: float = 0.6) -> np.ndarray:
    """Surface vertices at the start of `frame`: the input mesh rotated about the vertical
    axis through its centroid by omega t and translated by velocity t (t = frame dt), as
    float32 (a rigidly moving collision surface)."""
    v = np.asarray(verts, dtype=np.float64)
    t = frame * dt
    c = v.mean(axis=0)
    a = omega * t
    R = np.array([[math.cos(a), 0.0, math.sin(a)], [0.0, 1.0, 0.0],
                  [-math.sin(a), 0.0, math.cos(a)]])
    return ((v - c) @ R.T + c + np.asarray(velocity) * t).astype(np.float32)


def config(i: int, **kw):
    return [config0, config1, config2, config3, config4][i](**kw)
