"""Complex-step tangent of one cloth substep -- TEST INFRASTRUCTURE ONLY.

Forward-mode derivative J*delta of the substep map (x, v, k, c) -> (x', v') computed by the
complex-step method (Squire & Trapp 1998): every input gets an imaginary perturbation
i*eps*delta, the substep is evaluated in complex arithmetic, and Im(output)/eps is the
directional derivative, exact to rounding for eps ~ 1e-30 (no subtractive cancellation).

The substep is written out again here in numpy -- spring forces as in Alg. 1, semi-implicit
Euler with pins, contact response averaged over the hits of a node -- with the contact set
held at the one the real-valued step finds (or at given sets), which is how the adjoint
treats it.  It does not
call the C oracle's arithmetic except to list contact triangles, so it is an independent
check of the hand-written reverse-mode adjoint (``Model.substep_vjp``) through the identity
<J delta, lambda> = <delta, J^T lambda>.
"""
from __future__ import annotations

import numpy as np


def substep_jvp_cs(model, x, v, h, dx, dv, dk=None, dc=None, eps=1e-30, contacts=None):
    """Returns (x', v') real parts and (dx', dv') tangents of one substep at (x, v).
    contacts: node i's contact triangles as contacts[i] (held fixed whatever their distance);
    None = the sets the real-valued step finds."""
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    v = np.asarray(v, dtype=np.float64).reshape(-1, 3)
    N = x.shape[0]
    dk = np.zeros(model.S) if dk is None else np.asarray(dk, dtype=np.float64)
    dc = np.zeros(model.S) if dc is None else np.asarray(dc, dtype=np.float64)
    X = x + 1j * eps * np.asarray(dx, dtype=np.float64).reshape(-1, 3)
    V = v + 1j * eps * np.asarray(dv, dtype=np.float64).reshape(-1, 3)
    K = model.k + 1j * eps * dk
    Cd = model.c + 1j * eps * dc
    a, b = model.ends[:, 0], model.ends[:, 1]
    # spring forces (Alg. 1): dir = normalize(x_b - x_a); f = (k(|d| - L0) + c(v_b.dir - v_a.dir)) dir
    d = X[b] - X[a]
    length = np.sqrt(np.sum(d * d, axis=1))
    direction = d / length[:, None]
    spring = K * (length - model.rest)
    damp = Cd * (np.sum(V[b] * direction, axis=1) - np.sum(V[a] * direction, axis=1))
    f = (spring + damp)[:, None] * direction
    F = np.zeros((N, 3), dtype=np.complex128)
    np.add.at(F, a, f)
    np.add.at(F, b, -f)
    # semi-implicit Euler with pins
    free = model.w != 0.0
    Vs = np.where(free[:, None], V + h * (model.w[:, None] * F + model.g[None, :]), 0.0)
    Xs = np.where(free[:, None], X + h * Vs, X)
    # contact response with the real step's contact set
    if model.thickness > 0 and model.tris.shape[0] > 0:
        P = model.verts
        A = P[model.tris[:, 0]]
        nrm = np.cross(P[model.tris[:, 1]] - A, P[model.tris[:, 2]] - A)
        nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
        for i in np.nonzero(free)[0]:
            ids = (model.contacts(Xs[i].real) if contacts is None
                   else np.sort(np.asarray(contacts[i], dtype=np.int64)))
            if len(ids) == 0:
                continue
            push = model.thickness - np.sum((Xs[i][None, :] - A[ids]) * nrm[ids], axis=1)
            Xs[i] = Xs[i] + np.mean(push[:, None] * nrm[ids], axis=0)
            Vs[i] = -model.restitution * Vs[i]
    return Xs.real.copy(), Vs.real.copy(), Xs.imag / eps, Vs.imag / eps
