"""The one-substep parity checker accepts exactly the valid results: the oracle's own result,
either resolution of a near-threshold contact, and nothing perturbed."""
import numpy as np
import pytest

import oracle
from oracle.parity import substep_parity
from paper_2507_11794_amd import workloads as W


def test_accepts_oracle_result_and_rejects_perturbation():
    inp = W.small_collision_scene(n=14, freq=5, drop=0.165, spacing=0.02)
    m = oracle.Model.from_inputs(inp)
    x, v = m.run(inp.x0, inp.v0, inp.h, 200)
    x1, v1, cnt, _ = m.substep(x, v, inp.h)
    assert np.count_nonzero(cnt) > 0
    L = 0.26
    substep_parity(m, x, v, inp.h, x1, v1, L)
    i = int(np.nonzero(cnt)[0][0])
    bad = x1.copy()
    bad[i, 1] += 1e-5
    with pytest.raises(AssertionError):
        substep_parity(m, x, v, inp.h, bad, v1, L)
    badv = v1.copy()
    badv[i] *= -1.0  # contact ignored: velocity not reversed
    with pytest.raises(AssertionError):
        substep_parity(m, x, v, inp.h, x1, badv, L)


def test_rejects_a_substep_that_drops_the_damping():
    """The velocity bar is tight enough to see one substep taken without spring damping on
    the draped scene (the step differs from the true one by h w c |dv| per spring)."""
    inp = W.small_collision_scene(n=14, freq=5, drop=0.165, spacing=0.02)
    m = oracle.Model.from_inputs(inp)
    x, v = m.run(inp.x0, inp.v0, inp.h, 200)
    x1, v1, _, _ = m.substep(x, v, inp.h)
    undamped = oracle.Model.from_inputs(inp, c=np.zeros(inp.n_springs))
    x1b, v1b, _, _ = undamped.substep(x, v, inp.h)
    assert np.abs(v1b - v1).max() > 10 * 2e-5
    with pytest.raises(AssertionError):
        substep_parity(m, x, v, inp.h, x1b, v1b, 0.26)


def test_near_threshold_contact_accepts_both_resolutions_only():
    verts = np.array([[0, 0, 0], [1, 0, 0], [1, 0, 1], [0, 0, 1]], dtype=np.float64)
    tris = np.array([[0, 2, 1], [0, 3, 2]])
    th = 0.005
    m = oracle.Model(np.array([1e3]), np.zeros((0, 2)), [], [], [], gravity=(0, 0, 0),
                     verts=verts, tris=tris, thickness=th, cell=0.05)
    h = 1e-4
    x = np.array([[0.3, th + 2e-7, 0.6]])  # x* within 1e-6 of the threshold
    v = np.array([[0.2, 0.0, 0.1]])
    xs = x + h * v
    # no contact: x' = x*, v' = v*
    substep_parity(m, x, v, h, xs, v, 1.0)
    # contact: pushed to exactly th, velocity reversed and halved
    pushed = xs.copy()
    pushed[0, 1] = th
    substep_parity(m, x, v, h, pushed, -0.5 * v, 1.0)
    # mixed (pushed but velocity kept) is no valid resolution
    with pytest.raises(AssertionError):
        substep_parity(m, x, v, h, pushed, v + 0.1, 1.0)
