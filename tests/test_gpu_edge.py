"""Edge cases of the HIP path through the C ABI: a single node without springs landing on a
single triangle, a one-node-wide strip, a cloth of one wavefront plus one node (ragged last
wavefront) over a surface, a fully pinned cloth, a zero-frame step, and springs that all
have their own parameters.  Each is checked against the FP64 oracle (one substep at a time
where contacts occur) or against the exact invariant."""
import dataclasses

import numpy as np
import pytest

import oracle
from oracle.parity import substep_parity
from paper_2507_11794_amd import cloth as B
from paper_2507_11794_amd import workloads as W

pytestmark = pytest.mark.gpu


def h32(inp):
    return float(np.float32(np.float32(inp.dt) / np.float32(inp.n_substeps)))


def _floor(size=0.5, y=0.0):
    """One upward-facing triangle (counter-clockwise seen from +y) covering the origin."""
    verts = np.array([[-size, y, -size], [-size, y, 2 * size], [2 * size, y, -size]],
                     dtype=np.float32)
    return verts, np.array([[0, 1, 2]], dtype=np.int32)


def _scene(nx, ny, drop, spacing=0.01, pins=(), surface=True, n_steps=40, seed=3):
    rng = np.random.default_rng(seed)
    cloth = W.make_cloth(nx, ny, spacing, (0.0, drop, 0.0), W.K_STRUCT, W.K_SHEAR, W.K_BEND,
                         W.DAMPING, W.NODE_MASS, pins=list(pins), rng=rng)
    if not surface:
        return W._inputs(cloth, dt=1.0 / 600.0, n_substeps=4, n_steps=n_steps, name="edge")
    verts, tris = _floor()
    return W._inputs(cloth, verts, tris, thickness=0.005, cell_size=0.05, dt=1.0 / 600.0,
                     n_substeps=4, n_steps=n_steps, name="edge")


def _run_with_parity(inp, frames):
    """Step frame by frame, checking one substep against the oracle after every frame;
    returns the final state and the contacts seen."""
    model = oracle.Model.from_inputs(inp)
    L = max(float(np.max(np.ptp(inp.x0.astype(np.float64), axis=0))), 0.01)
    contacts = 0
    with B.Cloth(inp) as sim:
        for _ in range(frames):
            sim.step(n_steps=1)
            x, v = sim.read_state()
            sim.step(dt=h32(inp), n_substeps=1, n_steps=1)
            x1, v1 = sim.read_state()
            r = substep_parity(model, x, v, h32(inp), x1, v1, L, border=1e-6, tag="edge")
            contacts += r["contacts"]
        return sim.read_state(), contacts


def test_single_node_without_springs_lands_at_the_thickness():
    inp = _scene(1, 1, drop=0.02, n_steps=120)
    assert inp.ends.shape[0] == 0
    (x, v), contacts = _run_with_parity(inp, 120)
    assert contacts > 0
    # resting on the plane y = 0 at the thickness, up to one substep of gravity
    h = h32(inp)
    assert abs(float(x[0, 1]) - 0.005) <= 9.81 * h * h * 4


def test_strip_one_node_wide_matches_oracle_trajectory():
    inp = _scene(1, 37, drop=0.5, surface=False, pins=[(0, 0)], n_steps=50)
    with B.Cloth(inp) as sim:
        sim.step(n_steps=inp.n_steps)
        x, _ = sim.read_state()
    model = oracle.Model.from_inputs(inp)
    xr, _ = model.run(inp.x0, inp.v0, h32(inp), inp.n_steps * inp.n_substeps)
    side = float(np.max(np.ptp(inp.x0.astype(np.float64), axis=0)))
    assert np.abs(x.astype(np.float64) - xr).max() <= 1e-5 * side


def test_one_wavefront_plus_one_node_over_a_triangle():
    inp = _scene(13, 5, drop=0.012, spacing=0.008, n_steps=30)
    assert inp.n_nodes == 65
    _, contacts = _run_with_parity(inp, 30)
    assert contacts > 0


def test_fully_pinned_cloth_does_not_move():
    pins = [(r, c) for r in range(6) for c in range(7)]
    inp = _scene(7, 6, drop=0.003, pins=pins, n_steps=10)
    with B.Cloth(inp) as sim:
        sim.step(n_steps=10)
        x, v = sim.read_state()
    assert np.array_equal(x, inp.x0) and np.all(v == 0)


def test_zero_frames_leave_the_state_unchanged():
    inp = _scene(8, 8, drop=0.05, n_steps=5)
    with B.Cloth(inp) as sim:
        sim.step(n_steps=3)
        before = sim.read_state()
        sim.step(n_steps=0)
        after = sim.read_state()
    assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])


def test_every_spring_with_its_own_parameters():
    """Stiffness, damping and rest length drawn per spring, so the parameter table holds one
    entry per spring from the start: every frame's substep matches the oracle, and the
    one-substep and tile kernels agree bit for bit."""
    inp = _scene(24, 20, drop=0.012, n_steps=40, seed=11)
    rng = np.random.default_rng(12)
    S = inp.ends.shape[0]
    inp = dataclasses.replace(inp, k=(inp.k * rng.uniform(0.5, 1.0, S)).astype(np.float32),
                              c=(inp.c * rng.uniform(0.0, 2.0, S)).astype(np.float32),
                              rest=(inp.rest * rng.uniform(0.97, 1.03, S)).astype(np.float32))
    triples = set(zip(inp.k.tolist(), inp.c.tolist(), inp.rest.tolist()))
    assert len(triples) == S
    (x, v), contacts = _run_with_parity(inp, 30)
    print(f"{S} springs, {contacts} contacts")
    assert contacts > 0
    outs = []
    for kernel in (B.CLOTH_KERNEL_DIRECT, B.CLOTH_KERNEL_TILE, B.CLOTH_KERNEL_LANES2,
                   B.CLOTH_KERNEL_LANES4, B.CLOTH_KERNEL_GRID):
        with B.Cloth(inp) as sim:
            sim.set_launch(kernel=kernel)
            sim.step(n_steps=25)
            outs.append(sim.read_state())
    for x, v in outs[1:]:
        assert np.array_equal(outs[0][0], x) and np.array_equal(outs[0][1], v)


@pytest.mark.parametrize("shape", [(1, 37), (37, 1), (2, 2), (3, 5), (9, 17), (65, 3), (20, 20)])
def test_grid_kernel_on_ragged_shapes_equals_the_one_thread_kernel(shape):
    """The stencil kernel, with one and with two wavefronts per tile, on cloths whose sides are not multiples of the 8x8 tile (narrow
    last tile columns, short last tile rows, one-node-wide strips), over the floor triangle
    with a pinned corner: the same bits as the one-thread-per-node kernel after every frame,
    and its node order is the grid's tiles row by row."""
    nx, ny = shape
    inp = _scene(nx, ny, drop=0.012, spacing=0.008, pins=[(0, 0)], n_steps=30)
    outs = []
    for cfg in (dict(kernel=B.CLOTH_KERNEL_DIRECT, block_threads=64),
                dict(kernel=B.CLOTH_KERNEL_GRID, block_threads=64),
                dict(kernel=B.CLOTH_KERNEL_GRID, block_threads=128)):
        with B.Cloth(inp) as sim:
            sim.set_launch(**cfg)
            states = []
            for _ in range(inp.n_steps):
                sim.step(n_steps=1)
                states.append(sim.read_state())
            order = sim.node_order()
        outs.append(states)
    for other in outs[1:]:
        for (xa, va), (xb, vb) in zip(outs[0], other):
            assert np.array_equal(xa, xb) and np.array_equal(va, vb)
    want = [i * nx + j for tj in range(0, ny, 8) for ti in range(0, nx, 8)
            for i in range(tj, min(ny, tj + 8)) for j in range(ti, min(nx, ti + 8))]
    assert np.array_equal(order, want)


def test_grid_kernel_refused_for_springs_off_the_stencil():
    """A spring three columns long, or a second spring between the same two nodes, leaves
    the grid stencil: the grid kernel is refused (CLOTH_EINVAL) and the other kernels run."""
    base = _scene(6, 6, drop=0.02, n_steps=5)
    long_spring = dataclasses.replace(
        base, ends=np.concatenate([base.ends, [[0, 3]]]).astype(np.int32),
        rest=np.append(base.rest, np.float32(0.03)), k=np.append(base.k, np.float32(50.0)),
        c=np.append(base.c, np.float32(0.05)))
    doubled = dataclasses.replace(
        base, ends=np.concatenate([base.ends, base.ends[:1]]).astype(np.int32),
        rest=np.append(base.rest, base.rest[0]), k=np.append(base.k, base.k[0]),
        c=np.append(base.c, base.c[0]))
    for inp in (long_spring, doubled):
        with B.Cloth(inp) as sim:
            with pytest.raises(B.ClothError) as ei:
                sim.set_launch(kernel=B.CLOTH_KERNEL_GRID)
            assert ei.value.status == B.CLOTH_EINVAL
            sim.step(n_steps=5)
    with B.Cloth(base) as sim:
        sim.set_launch(kernel=B.CLOTH_KERNEL_GRID)
        sim.step(n_steps=5)


def test_read_state_fills_caller_arrays_and_round_trips_write_state():
    """cloth_read_state into caller-supplied arrays gives the same bits as into new ones,
    and a state written with cloth_write_state reads back exactly, in node-id order."""
    inp = _scene(13, 11, drop=0.012, n_steps=10)
    n = inp.n_nodes
    rng = np.random.default_rng(7)
    with B.Cloth(inp) as sim:
        sim.step(n_steps=10)
        x, v = sim.read_state()
        xo = np.full((n, 3), np.nan, np.float32)
        vo = np.full((n, 3), np.nan, np.float32)
        got = sim.read_state(xo, vo)
        assert got[0] is xo and got[1] is vo
        assert np.array_equal(x, xo) and np.array_equal(v, vo)
        xs = (inp.x0 + rng.normal(0.0, 1e-3, (n, 3))).astype(np.float32)
        vs = rng.normal(0.0, 0.1, (n, 3)).astype(np.float32)
        sim.write_state(xs, vs)
        x2, v2 = sim.read_state(xo, vo)
        assert np.array_equal(x2, xs) and np.array_equal(v2, vs)
