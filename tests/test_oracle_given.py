"""Pins for the oracle's fixed-contact-set entries, which the GPU adjoint tests use as their
reference: the substep, the rollout and the adjoint with given contact sets reduce to the
plain oracle step and adjoint when given the oracle's own sets (bit for bit), the given-set
adjoint is the transpose of an independent complex-step tangent for arbitrary fixed sets,
and the contact-set checker accepts exactly the valid sets.  Also pins the triangle-triangle
one-substep checker (mt_substep_parity)."""
import numpy as np
import pytest

import oracle
from oracle.parity import mt_substep_parity
from paper_2507_11794_amd import workloads as W


@pytest.fixture(scope="module")
def scene():
    inp = W.small_collision_scene(n=14, freq=5, drop=0.165, spacing=0.02)
    m = oracle.Model.from_inputs(inp)
    x, v = m.run(inp.x0, inp.v0, inp.h, 200)
    return inp, m, x, v


def own_sets(m, x, v, h):
    xp, _ = m.predict(x, v, h)
    return [m.contacts(xp[i]).tolist() if m.w[i] != 0 else [] for i in range(m.N)], xp


def test_scene_is_in_contact(scene):
    inp, m, x, v = scene
    sets, _ = own_sets(m, x, v, inp.h)
    assert sum(1 for s in sets if s) >= 5


def test_substep_given_own_sets_is_the_substep(scene):
    inp, m, x, v = scene
    sets, _ = own_sets(m, x, v, inp.h)
    x1, v1, _, _ = m.substep(x, v, inp.h)
    x2, v2 = m.substep_given(x, v, inp.h, sets)
    assert np.array_equal(x1, x2) and np.array_equal(v1, v2)


def test_run_given_own_sets_is_the_run(scene):
    inp, m, x, v = scene
    xs, vs, sets = x, v, []
    for _ in range(12):
        s, _ = own_sets(m, xs, vs, inp.h)
        sets.append(m.contact_csr(s))
        xs, vs, _, _ = m.substep(xs, vs, inp.h)
    xr, vr = m.run_given(x, v, inp.h, sets)
    assert np.array_equal(xr, xs) and np.array_equal(vr, vs)


def test_vjp_given_own_sets_is_the_vjp(scene):
    inp, m, x, v = scene
    rng = np.random.default_rng(3)
    lx, lv = rng.normal(size=(m.N, 3)), rng.normal(size=(m.N, 3))
    sets, _ = own_sets(m, x, v, inp.h)
    a = m.substep_vjp(x, v, inp.h, lx, lv)
    b = m.substep_vjp_given(x, v, inp.h, sets, lx, lv)
    for p, q in zip(a, b):
        assert np.array_equal(p, q)
    # the sets matter: dropping one contact changes that node's adjoint
    i = next(i for i, s in enumerate(sets) if s)
    dropped = [list(s) for s in sets]
    dropped[i] = dropped[i][1:]
    c = m.substep_vjp_given(x, v, inp.h, dropped, lx, lv)
    assert np.abs(c[0][i] - a[0][i]).max() > 1e-6


@pytest.mark.parametrize("variant", ["own", "dropped", "extra", "every_node"])
def test_vjp_given_is_transpose_of_complex_step_tangent(scene, variant):
    """<J d, l> = <d, J^T l> for the substep with fixed sets, including sets that are not
    the step's own (a dropped contact, an extra far triangle, a node with several)."""
    inp, m, x, v = scene
    sets, _ = own_sets(m, x, v, inp.h)
    rng = np.random.default_rng({"own": 0, "dropped": 1, "extra": 2, "every_node": 3}[variant])
    contact_nodes = [i for i, s in enumerate(sets) if s]
    if variant == "dropped":
        for i in contact_nodes[::2]:
            sets[i] = sets[i][:-1]
    elif variant == "extra":
        for i in range(0, m.N, 7):
            extra = int(rng.integers(0, m.tris.shape[0]))
            sets[i] = sorted(set(sets[i]) | {extra})
    elif variant == "every_node":
        sets = [sorted(set(s) | {int(t)}) for s, t in
                zip(sets, rng.integers(0, m.tris.shape[0], size=m.N))]
    N, S = m.N, m.S
    dx, dv = rng.normal(size=(N, 3)), rng.normal(size=(N, 3))
    dk, dc = rng.normal(size=S) * 50, rng.normal(size=S) * 0.01
    lx, lv = rng.normal(size=(N, 3)), rng.normal(size=(N, 3))
    xr, vr, tx, tv = oracle.substep_jvp_cs(m, x, v, inp.h, dx, dv, dk, dc, contacts=sets)
    x1, v1 = m.substep_given(x, v, inp.h, sets)
    assert np.abs(xr - x1).max() <= 1e-14 and np.abs(vr - v1).max() <= 1e-12
    xb, vb, kb, cb = m.substep_vjp_given(x, v, inp.h, sets, lx, lv)
    lhs = np.sum(tx * lx) + np.sum(tv * lv)
    rhs = np.sum(dx * xb) + np.sum(dv * vb) + np.sum(dk * kb) + np.sum(dc * cb)
    scale = np.abs(tx * lx).sum() + np.abs(tv * lv).sum()
    assert abs(lhs - rhs) <= 1e-10 * scale


def test_contact_checker_accepts_exactly_the_valid_sets(scene):
    inp, m, x, v = scene
    sets, xp = own_sets(m, x, v, inp.h)
    st, nb = m.check_contacts(xp, sets, 1e-6)
    assert not st.any()
    i = next(i for i, s in enumerate(sets) if s)
    # a sure contact missing
    bad = [list(s) for s in sets]
    bad[i] = bad[i][1:]
    st, _ = m.check_contacts(xp, bad, 1e-6)
    assert st[i] == 2 and np.count_nonzero(st) == 1
    # a far triangle listed
    far = next(t for t in range(m.tris.shape[0])
               if np.sqrt(oracle.point_tri_dist2(xp[i], *m.verts[m.tris[t]])) > 0.05)
    bad = [list(s) for s in sets]
    bad[i] = sorted(bad[i] + [far])
    st, _ = m.check_contacts(xp, bad, 1e-6)
    assert st[i] == 1 and np.count_nonzero(st) == 1


def test_contact_checker_border_decisions():
    """A node whose distance lies within the border of the thickness may list the triangle
    or not; just outside the border only one decision is valid."""
    verts = np.array([[0, 0, 0], [1, 0, 0], [1, 0, 1], [0, 0, 1]], dtype=np.float64)
    tris = np.array([[0, 2, 1], [0, 3, 2]])
    th = 0.005
    m = oracle.Model(np.array([1e3, 1e3, 0.0]), np.zeros((0, 2)), [], [], [], gravity=(0, 0, 0),
                     verts=verts, tris=tris, thickness=th, cell=0.05)
    xp = np.array([[0.3, th + 2e-7, 0.6], [0.7, th - 3e-6, 0.2], [0.5, 0.001, 0.5]])
    t0 = 0 if np.sqrt(oracle.point_tri_dist2(xp[0], *verts[tris[0]])) < 0.01 else 1
    t1 = 0 if np.sqrt(oracle.point_tri_dist2(xp[1], *verts[tris[0]])) < 0.01 else 1
    ok_sets = ([[t0], [t1], []], [[], [t1], []])
    for s in ok_sets:
        st, _ = m.check_contacts(xp, s, 1e-6)
        assert not st.any(), s
    st, nb = m.check_contacts(xp, ok_sets[0], 1e-6)
    assert nb == 1
    st, _ = m.check_contacts(xp, [[], [], []], 1e-6)  # node 1 is 3e-6 inside: must list
    assert st.tolist() == [0, 2, 0]
    st, _ = m.check_contacts(xp, [[], [t1], [0]], 1e-6)  # pinned node never collides
    assert st.tolist() == [0, 0, 3]


def test_mt_checker_accepts_oracle_step_and_rejects_perturbation():
    inp = W.small_collision_scene(n=16, n_steps=90)
    m = oracle.Model.from_inputs(inp)
    h = inp.h
    x, v = inp.x0.astype(np.float64), inp.v0.astype(np.float64)
    hit = None
    for _ in range(90 * inp.n_substeps):
        x1, v1, cnt, _ = m.substep_mt(inp.nx, inp.ny, x, v, h)
        if np.count_nonzero(cnt) >= 3:
            hit = (x, v, x1, v1, cnt)
            break
        x, v = x1, v1
    assert hit is not None, "the scene never reached the surface"
    x, v, x1, v1, cnt = hit
    L = float(np.max(np.ptp(inp.x0.astype(np.float64), axis=0)))
    mt_substep_parity(m, inp.nx, inp.ny, x, v, h, x1, v1, L)
    i = int(np.nonzero(cnt)[0][0])
    bad = x1.copy()
    bad[i, 1] += 1e-5
    with pytest.raises(AssertionError):
        mt_substep_parity(m, inp.nx, inp.ny, x, v, h, bad, v1, L)
    badv = v1.copy()
    badv[i] *= -1.0
    with pytest.raises(AssertionError):
        mt_substep_parity(m, inp.nx, inp.ny, x, v, h, x1, badv, L)
    # ignoring the contacts (the prediction kept) is no valid result either
    xs, vs = m.predict(x, v, h)
    with pytest.raises(AssertionError):
        mt_substep_parity(m, inp.nx, inp.ny, x, v, h, xs, vs, L)
