"""One-substep parity check of a device result against the oracle -- TEST INFRASTRUCTURE.

A contact is decided by comparing a point-triangle distance with the thickness.  When the
FP64 distance lies within ``border`` of the thickness, FP32 arithmetic may legitimately take
either decision, and after a push the node sits at exactly the thickness from the pushing
triangle's plane, so such near-threshold decisions are common.  Nodes with such a triangle
are therefore checked against every valid resolution: the oracle's response with the sure
contacts plus any subset of the ambiguous ones must reproduce the device result.
"""
from __future__ import annotations

import itertools

import numpy as np

# Bars of a one-substep comparison of an FP32 result with the FP64 oracle.  Positions: 1e-6
# of the cloth's extent L per coordinate; an FP32 coordinate of a ~1 m cloth rounds to
# ~6e-8 m, and the measured worst clean-node error on the 316x316 workload is 3.0e-8 L.  Velocities: 2e-5 m/s plus 1e-5 of the largest speed; the spring
# force sums about twelve differences of FP32 positions, and h w F moves v by a few 1e-7 m/s
# (measured worst 7.9e-7 m/s on the 316x316 workload, 5.9e-7 m/s on the 800x800 cloth),
# while dropping a spring's damping for one substep moves it by h w c |dv| = 2e-2 |dv| at
# the workloads' h, w, c, i.e. above the bar wherever neighbours' velocities differ by more
# than about 1e-3 m/s.
XTOL = 1e-6
VTOL_ABS = 2e-5
VTOL_REL = 1e-5


def substep_parity(model, x, v, h, x1, v1, L, border=1e-6, xtol=XTOL, vtol_abs=VTOL_ABS,
                   vtol_rel=VTOL_REL, tag=""):
    """Raises AssertionError on a mismatch; returns summary statistics.

    x, v: the state the device started from (FP32 arrays, [N,3]); x1, v1: the device's state
    one substep of length h later; L: length scale for the position tolerance xtol * L."""
    x64, v64 = np.asarray(x, np.float64), np.asarray(v, np.float64)
    xr, vr, cnt, margin = model.substep(x64, v64, h)
    X1, V1 = np.asarray(x1, np.float64), np.asarray(v1, np.float64)
    ex = np.abs(X1 - xr).max(axis=1)
    ev = np.abs(V1 - vr).max(axis=1)
    vtol = vtol_abs + vtol_rel * float(np.abs(vr).max())
    amb = margin < border
    bad = np.nonzero(~amb & ((ex > xtol * L) | (ev > vtol)))[0]
    assert bad.size == 0, (tag, "mismatch", bad[:8].tolist(), ex[bad[:8]].tolist(),
                           ev[bad[:8]].tolist())
    resolved = 0
    if amb.any():
        xs, vs = model.predict(x64, v64, h)
        th = model.thickness
        for i in np.nonzero(amb)[0]:
            ids, dist = model.box_candidates(xs[i])
            sure = [int(t) for t, d in zip(ids, dist) if d < th - border]
            maybe = [int(t) for t, d in zip(ids, dist) if abs(d - th) <= border]
            assert len(maybe) <= 10, (tag, "too many ambiguous contacts", i, len(maybe))
            ok = False
            for r in range(len(maybe) + 1):
                for sub in itertools.combinations(maybe, r):
                    p, q = model.respond(xs[i], vs[i], sorted(sure + list(sub)))
                    if (np.abs(p - X1[i]).max() <= xtol * L and np.abs(q - V1[i]).max() <= vtol):
                        ok = True
                        break
                if ok:
                    break
            assert ok, (tag, "ambiguous node matches no valid resolution", int(i), sure, maybe,
                        X1[i].tolist(), xr[i].tolist())
            resolved += 1
    clean = ~amb
    return dict(contacts=int(np.count_nonzero(cnt)), ambiguous=int(amb.sum()),
                resolved=resolved, ex=float(ex[clean].max() / L) if clean.any() else 0.0,
                ev=float(ev[clean].max()) if clean.any() else 0.0)


def resolve_contacts(model, x, v, h, x1, v1, L, border=1e-6, xtol=XTOL, vtol_abs=VTOL_ABS,
                     vtol_rel=VTOL_REL):
    """The contact set another implementation used in one substep from (x, v) to (x1, v1):
    per node, the oracle's sure contacts plus the subset of near-threshold triangles whose
    response reproduces (x1, v1).  Raises AssertionError if no valid set does."""
    x64, v64 = np.asarray(x, np.float64), np.asarray(v, np.float64)
    X1, V1 = np.asarray(x1, np.float64), np.asarray(v1, np.float64)
    xs, vs = model.predict(x64, v64, h)
    th = model.thickness
    vtol = vtol_abs + vtol_rel * float(np.abs(vs).max())
    out = []
    for i in range(x64.shape[0]):
        if model.w[i] == 0.0 or th <= 0:
            out.append([])
            continue
        ids, dist = model.box_candidates(xs[i])
        sure = [int(t) for t, d in zip(ids, dist) if d < th - border]
        maybe = [int(t) for t, d in zip(ids, dist) if abs(d - th) <= border]
        found = None
        for r in range(len(maybe) + 1):
            for sub in itertools.combinations(maybe, r):
                cs = sorted(sure + list(sub))
                p, q = model.respond(xs[i], vs[i], cs)
                if np.abs(p - X1[i]).max() <= xtol * L and np.abs(q - V1[i]).max() <= vtol:
                    found = cs
                    break
            if found is not None:
                break
        assert found is not None, ("no contact set reproduces node", i)
        out.append(found)
    return out


def mt_substep_parity(model, nx, ny, x, v, h, x1, v1, L, border=2e-6, xtol=XTOL,
                      vtol_abs=VTOL_ABS, vtol_rel=VTOL_REL, tag=""):
    """substep_parity for the triangle-triangle narrow phase: nodes whose tests all lie at
    least ``border`` from a decision boundary must match the oracle's substep; the others
    must match the response to the sure contacts plus some subset of the near-boundary
    candidates."""
    x64, v64 = np.asarray(x, np.float64), np.asarray(v, np.float64)
    xr, vr, cnt, margin = model.substep_mt(nx, ny, x64, v64, h)
    X1, V1 = np.asarray(x1, np.float64), np.asarray(v1, np.float64)
    ex = np.abs(X1 - xr).max(axis=1)
    ev = np.abs(V1 - vr).max(axis=1)
    vtol = vtol_abs + vtol_rel * float(np.abs(vr).max())
    amb = margin < border
    bad = np.nonzero(~amb & ((ex > xtol * L) | (ev > vtol)))[0]
    assert bad.size == 0, (tag, "mismatch", bad[:8].tolist(), ex[bad[:8]].tolist(),
                           ev[bad[:8]].tolist(), cnt[bad[:8]].tolist())
    if amb.any():
        xs, vs = model.predict(x64, v64, h)
        for i in np.nonzero(amb)[0]:
            ids, hits, mg = model.mt_candidates(nx, ny, x64, xs, i)
            sure = [int(t) for t, hh, g in zip(ids, hits, mg) if hh and g >= border]
            maybe = [int(t) for t, g in zip(ids, mg) if g < border]
            assert len(maybe) <= 10, (tag, "too many ambiguous candidates", int(i), len(maybe))
            ok = False
            for r in range(len(maybe) + 1):
                for sub in itertools.combinations(maybe, r):
                    p, q = model.respond(xs[i], vs[i], sorted(sure + list(sub)))
                    if np.abs(p - X1[i]).max() <= xtol * L and np.abs(q - V1[i]).max() <= vtol:
                        ok = True
                        break
                if ok:
                    break
            assert ok, (tag, "ambiguous node matches no valid resolution", int(i), sure, maybe)
    clean = ~amb
    return dict(contacts=int(np.count_nonzero(cnt)), ambiguous=int(amb.sum()),
                ex=float(ex[clean].max() / L) if clean.any() else 0.0)
