"""Point-in-closed-surface test for whole cloth states -- TEST INFRASTRUCTURE ONLY.

A point p is inside a closed triangle surface iff the segment from a point o known to be
inside crosses the surface an even number of times (the crossing number of the segment
o -> p, counted with the Moller-Trumbore segment-triangle intersection).  Every crossing of
that segment lies in direction (p - o)/|p - o| seen from o, so only triangles whose angular
extent seen from o contains that direction can be crossed: they are found with a k-d tree
over the triangles' centroid directions (search radius = the largest chord between a
triangle's centroid direction and its vertices' directions), which makes the test fast
enough for 100K points against 100K triangles.
"""
from __future__ import annotations

import numpy as np


def inside_closed_mesh(P, V, F, origin=(1.37e-5, -2.11e-5, 0.73e-5), chunk=4096):
    """Boolean [n]: P[i] strictly inside the closed surface (V, F); origin must be inside and
    every triangle must subtend less than a half sphere from it.  The default origin sits a
    few tens of micrometres off the centre of the workloads' spheres, so segments do not run
    through mesh vertices or edges along the radial lines the meshes are built on."""
    from scipy.spatial import cKDTree

    P = np.asarray(P, dtype=np.float64).reshape(-1, 3)
    o = np.asarray(origin, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64) - o
    F = np.asarray(F, dtype=np.int64)
    A, B, C = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    unit = lambda a: a / np.linalg.norm(a, axis=-1, keepdims=True)  # noqa: E731
    cen = unit(A + B + C)
    rad = np.max([np.linalg.norm(cen - unit(X), axis=1) for X in (A, B, C)], axis=0)
    tree = cKDTree(cen)
    e1, e2 = B - A, C - A
    Q = P - o
    # a point beyond the farthest vertex lies outside the surface's bounding ball
    near = np.nonzero(np.linalg.norm(Q, axis=1) <= np.linalg.norm(V, axis=1).max())[0]
    inside = np.zeros(P.shape[0], dtype=bool)
    if near.size < P.shape[0]:
        inside[near] = inside_closed_mesh(Q[near], V, F, (0.0, 0.0, 0.0), chunk) if near.size else False
        return inside
    dirs = unit(Q + 1e-300)
    r_search = float(rad.max()) * 1.0001 + 1e-12
    for s in range(0, P.shape[0], chunk):
        cand = tree.query_ball_point(dirs[s:s + chunk], r_search)
        rows = np.repeat(np.arange(s, s + len(cand)), [len(c) for c in cand])
        tris = np.fromiter((t for c in cand for t in c), dtype=np.int64, count=rows.size)
        if rows.size == 0:
            continue
        d = Q[rows]                      # segment o -> p, parameter t in (0, 1)
        a_, ee1, ee2 = A[tris], e1[tris], e2[tris]
        h = np.cross(d, ee2)
        a = np.einsum("ij,ij->i", ee1, h)
        ok = np.abs(a) > 1e-300
        f = np.where(ok, 1.0 / np.where(ok, a, 1.0), 0.0)
        sv = -a_                          # o - A (o is the new origin)
        u = f * np.einsum("ij,ij->i", sv, h)
        q = np.cross(sv, ee1)
        v = f * np.einsum("ij,ij->i", d, q)
        t = f * np.einsum("ij,ij->i", ee2, q)
        hit = ok & (u >= 0) & (v >= 0) & (u + v <= 1) & (t > 0) & (t < 1)
        crossings = np.bincount(rows[hit] - s, minlength=len(cand))
        inside[s:s + len(cand)] = crossings % 2 == 0
    return inside
