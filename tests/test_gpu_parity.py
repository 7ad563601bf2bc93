"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same seeded
inputs.

Tolerances.  FP32 rounds positions of ~1 m magnitude to ~6e-8 m; one substep moves a node by
h v* with v* carrying the spring-force rounding (differences of FP32 positions, ~1e-7
relative) scaled by h w, so one-substep positions agree to about an ulp of the coordinates
(bar: 1e-6 of the cloth side; measured worst 3.0e-8 on the 316x316 workload) and velocities
to a few 1e-7 m/s (bar: 2e-5 m/s plus 1e-5 of the largest speed; measured worst 7.9e-7 m/s),
the bars of oracle/parity.py.  Over 100 frames of the collision-free hanging cloth the FP32 trajectory
must stay within 1e-5 of the cloth side length.  A contact decision with |dist - th| within
1e-6 m of the threshold may legitimately differ between FP32 and FP64; such nodes are
checked against every valid resolution of their near-threshold triangles.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from oracle.parity import substep_parity
from paper_2507_11794_amd import cloth as B
from paper_2507_11794_amd import workloads as W

pytestmark = pytest.mark.gpu

BORDER = 1e-6


def h32(inp, n_substeps=None):
    ns = inp.n_substeps if n_substeps is None else n_substeps
    return float(np.float32(np.float32(inp.dt) / np.float32(ns)))


def side(inp):
    return float(np.max(np.ptp(inp.x0.astype(np.float64), axis=0)))


def one_substep_check(inp, x, v, x1, v1, model, tag=""):
    """Oracle substep from the GPU state (x, v) versus the GPU's own next state (x1, v1);
    near-threshold contact decisions are checked against every valid resolution."""
    return substep_parity(model, x, v, h32(inp), x1, v1, side(inp), border=BORDER, tag=tag)


def test_config0_trajectory_within_1e5_after_100_frames():
    inp = W.config0()
    with B.Cloth(inp) as sim:
        sim.step(n_steps=inp.n_steps)
        x, v = sim.read_state()
    model = oracle.Model.from_inputs(inp)
    xr, vr = model.run(inp.x0, inp.v0, h32(inp), inp.n_steps * inp.n_substeps)
    err = np.abs(x.astype(np.float64) - xr).max() / side(inp)
    print(f"config0 100 frames: max |x_gpu - x_oracle| / L = {err:.3e}")
    assert err <= 1e-5
    # pinned nodes never move
    pins = inp.pinned.astype(bool)
    assert np.array_equal(x[pins], inp.x0[pins]) and np.all(v[pins] == 0)


def test_bitwise_deterministic_runs():
    inp = W.config0()
    outs = []
    for _ in range(2):
        with B.Cloth(inp) as sim:
            sim.step(n_steps=25)
            outs.append(sim.read_state())
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_resume_is_bit_exact():
    inp = W.small_collision_scene(n=24, n_steps=60)
    with B.Cloth(inp) as a:
        a.step(n_steps=60)
        xa, va = a.read_state()
    with B.Cloth(inp) as b:
        b.step(n_steps=25)
        xs, vs = b.read_state()
    with B.Cloth(inp) as c:
        c.write_state(xs, vs)
        c.step(n_steps=35)
        xc, vc = c.read_state()
    assert np.array_equal(xa, xc) and np.array_equal(va, vc)


def _tiny_surfaces():
    yield W.small_collision_scene(n=8, freq=3)
    yield W.small_collision_scene(n=8, freq=6)
    c1 = W.config1(n=20, freq=4)
    yield c1
    # a grid of more cells than a workgroup can count in LDS, with the triangles in a random
    # order: every workgroup's cell box spans the grid, so the build takes its global-atomic
    # path (the surface in mesh order takes the LDS path)
    c2 = W.config1(n=20, freq=24)
    yield c2
    perm = np.random.default_rng(5).permutation(c2.tris.shape[0])
    yield dataclasses.replace(c2, tris=np.ascontiguousarray(c2.tris[perm]))


@pytest.mark.parametrize("which", [0, 1, 2, 3, 4])
def test_broadphase_candidates_equal_fp32_brute_force(which):
    """The step kernels' own query (coded box test of the point's cell, undecided boxes
    settled with the exact box, through the LDS hit list or, when it overflows or is off,
    the unlisted loop) against the O(points x triangles) FP32 brute force, bit for bit, on
    random points, points outside the grid, points on and one ulp either side of inflated
    box faces, points within a few 1/32768 of a cell width of box faces (where the coded
    test is undecided) and points on grid-cell faces."""
    inp = list(_tiny_surfaces())[which]
    rng = np.random.default_rng(100 + which)
    V = inp.verts.astype(np.float64)
    th = np.float32(inp.thickness)
    cell = np.float32(inp.cell_size)
    pts = [V[rng.integers(0, V.shape[0], 1500)] + rng.normal(0, 0.008, size=(1500, 3))]
    # far outside the grid
    pts.append(rng.uniform(-3, 3, size=(200, 3)))
    T = inp.tris
    lo = np.min(inp.verts[T], axis=1) - th
    hi = np.max(inp.verts[T], axis=1) + th
    pick = rng.integers(0, T.shape[0], 200)
    base = (lo[pick] + hi[pick]) * np.float32(0.5)
    for bound in (lo[pick], hi[pick]):
        for axis in range(3):
            # exactly on, and 1-3 ulps either side of, the face
            for d in (-3, -2, -1, 0, 1, 2, 3):
                q = base.copy()
                q[:, axis] = bound[:, axis]
                for _ in range(abs(d)):
                    q[:, axis] = np.nextafter(q[:, axis], np.float32(np.sign(d) * np.inf))
                pts.append(q.astype(np.float64))
            # within a few code buckets (1/32768 of a cell) of the face
            for f in (-2.0, -1.0, -0.5, -0.25, 0.25, 0.5, 1.0, 2.0):
                q = base.copy()
                q[:, axis] = bound[:, axis] + np.float32(f / 32768.0) * cell
                pts.append(q.astype(np.float64))
    # on grid-cell faces (origin min(V) - thickness, as the grid is built) and one ulp away
    org = np.min(inp.verts, axis=0) - th
    q0 = (V[rng.integers(0, V.shape[0], 300)] + rng.normal(0, 0.004, size=(300, 3))).astype(np.float32)
    for axis in range(3):
        for d in (-1, 0, 1):
            q = q0.copy()
            k = np.round((q[:, axis] - org[axis]) / cell)
            q[:, axis] = (org[axis] + k * cell).astype(np.float32)
            if d:
                q[:, axis] = np.nextafter(q[:, axis], np.float32(d * np.inf))
            pts.append(q.astype(np.float64))
    P = np.concatenate(pts).astype(np.float32)
    want = oracle.candidates_f32(P, inp.verts, inp.tris, inp.thickness)
    with B.Cloth(inp) as sim:
        info = sim.info()
        assert info["cells"] > 0
        for slots in (32, 2, 0):  # default list, lists that overflow, no list
            sim.set_launch(hit_slots=slots)
            got = sim.debug_candidates(P)
            print(f"surface {which}, hit_slots {slots}: {P.shape[0]} points, "
                  f"{want.shape[0]} pairs, grid {info}")
            assert got.shape == want.shape and np.array_equal(got, want), slots


def test_one_substep_parity_with_collision_small():
    inp = W.small_collision_scene(n=24, n_steps=120)
    model = oracle.Model.from_inputs(inp)
    total_contacts, total_amb = 0, 0
    with B.Cloth(inp) as sim:
        for frame in range(inp.n_steps):
            x, v = sim.read_state()
            sim.step(dt=h32(inp), n_substeps=1, n_steps=1)
            x1, v1 = sim.read_state()
            if frame % 3 == 0 or frame > 60:
                r = one_substep_check(inp, x, v, x1, v1, model, tag=f"substep {frame}")
                total_contacts += r["contacts"]
                total_amb += r["ambiguous"]
            sim.step(dt=h32(inp), n_substeps=1, n_steps=inp.n_substeps - 1)
    print(f"contacts {total_contacts}, near-threshold nodes resolved {total_amb}")
    assert total_contacts > 500


def test_config1_whole_run_parity_and_no_penetration():
    """The 316x316 cloth dropped on the 100,820-triangle sphere, 300 frames: one substep
    checked against the oracle from the GPU's own state at frame 0 and every 10th frame
    (near-threshold contacts resolved), and no node inside the closed surface after every
    5th frame and after every substep of frames 100-101 (the surface is never penetrated,
    Sec. 4.2).  The largest position and velocity errors of the clean nodes are printed."""
    from oracle.inside import inside_closed_mesh

    inp = W.config1()
    model = oracle.Model.from_inputs(inp)
    h = h32(inp)
    worst_x = worst_v = 0.0
    contacts = amb = checked = inside_checks = 0
    with B.Cloth(inp) as sim:
        for frame in range(inp.n_steps):
            if frame % 10 == 0 or frame == inp.n_steps - 1:
                x, v = sim.read_state()
                sim.step(dt=h, n_substeps=1, n_steps=1)
                x1, v1 = sim.read_state()
                r = one_substep_check(inp, x, v, x1, v1, model, tag=f"config1 frame {frame}")
                worst_x, worst_v = max(worst_x, r["ex"]), max(worst_v, r["ev"])
                contacts += r["contacts"]
                amb += r["ambiguous"]
                checked += 1
                sim.step(dt=h, n_substeps=1, n_steps=inp.n_substeps - 1)
            elif frame in (100, 101):
                for _ in range(inp.n_substeps):
                    sim.step(dt=h, n_substeps=1, n_steps=1)
                    x, _ = sim.read_state()
                    assert not inside_closed_mesh(x, inp.verts, inp.tris).any(), frame
                    inside_checks += 1
            else:
                sim.step(n_steps=1)
            if frame % 50 == 49:
                print(f"  config1 frame {frame + 1}: {checked} substeps checked", flush=True)
            if frame % 5 == 4:
                x, _ = sim.read_state()
                bad = np.nonzero(inside_closed_mesh(x, inp.verts, inp.tris))[0]
                assert bad.size == 0, ("penetration after frame", frame, bad[:8].tolist())
                inside_checks += 1
    print(f"config1: {checked} substeps checked, {contacts} contacts, {amb} near-threshold "
          f"nodes resolved; worst clean-node error |dx|/L = {worst_x:.2e}, |dv| = "
          f"{worst_v:.2e} m/s; {inside_checks} no-penetration checks")
    assert contacts > 10000


def test_config2_full_size_one_substep_parity():
    inp = W.config2()
    model = oracle.Model.from_inputs(inp)
    with B.Cloth(inp) as sim:
        sim.step(n_steps=20)
        x, v = sim.read_state()
        sim.step(dt=h32(inp), n_substeps=1, n_steps=1)
        x1, v1 = sim.read_state()
    r = one_substep_check(inp, x, v, x1, v1, model, tag="config2")
    print(f"config2: {r}")


def test_unstable_substep_rejected():
    inp = W.config0()
    with B.Cloth(inp) as sim:
        with pytest.raises(B.ClothError) as ei:
            sim.step(dt=1.0 / 600, n_substeps=1, n_steps=1)
        assert ei.value.status == B.CLOTH_EUNSTABLE


def test_nan_flag_reported():
    inp = W.config0(n=8)
    with B.Cloth(inp, flags=B.CLOTH_F_CHECK_NAN | B.CLOTH_F_NO_STABILITY_CHECK) as sim:
        sim.step(dt=0.5, n_substeps=1, n_steps=30)  # far beyond the stability limit
        with pytest.raises(B.ClothError) as ei:
            sim.read_state()
        assert ei.value.status == B.CLOTH_ENAN


LAUNCHES = [
    dict(kernel=B.CLOTH_KERNEL_DIRECT, block_threads=64, use_graph=0, split_refs=0),
    dict(kernel=B.CLOTH_KERNEL_DIRECT, block_threads=256, use_graph=1, hit_slots=0, split_refs=0),
    dict(kernel=B.CLOTH_KERNEL_DIRECT, block_threads=64, use_graph=1, split_refs=8),
    dict(kernel=B.CLOTH_KERNEL_DIRECT, block_threads=128, use_graph=0, split_refs=1, hit_slots=2),
    dict(kernel=B.CLOTH_KERNEL_DIRECT, block_threads=128, use_graph=1, hit_slots=4, xcd_runs=1),
    dict(kernel=B.CLOTH_KERNEL_DIRECT, block_threads=64, use_graph=1, xcd_runs=3),
    dict(kernel=B.CLOTH_KERNEL_DIRECT, block_threads=256, use_graph=0, xcd_runs=16),
    dict(kernel=B.CLOTH_KERNEL_TILE, tile_nodes=64, substeps_per_launch=1, use_graph=0),
    dict(kernel=B.CLOTH_KERNEL_TILE, tile_nodes=256, substeps_per_launch=2, use_graph=1),
    dict(kernel=B.CLOTH_KERNEL_TILE, tile_nodes=256, substeps_per_launch=3, use_graph=1),
    dict(kernel=B.CLOTH_KERNEL_TILE, tile_nodes=1024, substeps_per_launch=4, block_threads=128,
         use_graph=1),
    dict(kernel=B.CLOTH_KERNEL_TILE, tile_nodes=128, substeps_per_launch=8, use_graph=0),
    dict(kernel=B.CLOTH_KERNEL_LANES2, block_threads=64, use_graph=1, hit_slots=8),
    dict(kernel=B.CLOTH_KERNEL_LANES2, block_threads=256, use_graph=0, hit_slots=0, xcd_runs=3),
    dict(kernel=B.CLOTH_KERNEL_LANES4, block_threads=64, use_graph=1, hit_slots=8),
    dict(kernel=B.CLOTH_KERNEL_LANES4, block_threads=128, use_graph=1, hit_slots=1),
    dict(kernel=B.CLOTH_KERNEL_LANES4, block_threads=256, use_graph=0, hit_slots=0, xcd_runs=1),
    dict(kernel=B.CLOTH_KERNEL_GRID, block_threads=64, use_graph=1),
    dict(kernel=B.CLOTH_KERNEL_GRID, block_threads=64, use_graph=0, hit_slots=0),
    dict(kernel=B.CLOTH_KERNEL_GRID, block_threads=64, use_graph=1, hit_slots=4, xcd_runs=3),
    dict(kernel=B.CLOTH_KERNEL_GRID, block_threads=128, use_graph=1),
    dict(kernel=B.CLOTH_KERNEL_GRID, block_threads=128, use_graph=0, hit_slots=0),
    dict(kernel=B.CLOTH_KERNEL_GRID, block_threads=128, use_graph=1, hit_slots=4, xcd_runs=3),
    dict(kernel=B.CLOTH_KERNEL_GRID, block_threads=256, use_graph=1, hit_slots=64, xcd_runs=16),
]


@pytest.mark.parametrize("scene", ["small", "config1_64"])
def test_every_launch_configuration_is_bit_identical(scene):
    if scene == "small":
        inp = W.small_collision_scene(n=40, n_steps=90, spacing=0.008)
    else:
        inp = W.config1(n=64, freq=20, n_steps=150)
    outs = []
    for cfg in LAUNCHES:
        with B.Cloth(inp) as sim:
            sim.set_launch(**cfg)
            # an odd substep count exercises the remainder launch and graph parity
            sim.step(n_steps=inp.n_steps)
            sim.step(dt=h32(inp), n_substeps=1, n_steps=3)
            outs.append((cfg, *sim.read_state()))
    ref = outs[0]
    for cfg, x, v in outs[1:]:
        assert np.array_equal(x, ref[1]) and np.array_equal(v, ref[2]), cfg
    moved = np.abs(ref[1] - inp.x0).max()
    assert moved > 0.01


@pytest.mark.parametrize("kernel", [B.CLOTH_KERNEL_GRID, B.CLOTH_KERNEL_DIRECT,
                                    B.CLOTH_KERNEL_TILE])
def test_default_and_tile_kernels_match_oracle_one_substep(kernel):
    inp = W.config1(n=96, freq=24)
    model = oracle.Model.from_inputs(inp)
    with B.Cloth(inp) as sim:
        if kernel == B.CLOTH_KERNEL_GRID:
            # the default for one grid cloth with a surface: two wavefronts per tile
            assert sim.get_launch()["kernel"] == B.CLOTH_KERNEL_GRID
            assert sim.get_launch()["block_threads"] == 128
        else:
            sim.set_launch(kernel=kernel, block_threads=256 if kernel == B.CLOTH_KERNEL_TILE else 64)
        sim.step(n_steps=120)
        for _ in range(3):
            x, v = sim.read_state()
            sim.step(dt=h32(inp), n_substeps=1, n_steps=1)
            x1, v1 = sim.read_state()
            r = one_substep_check(inp, x, v, x1, v1, model, tag="tile default")
    assert r["contacts"] > 100


def _sliver_fan_scene(n_fan=400, n=24, spacing=0.008, drop=0.02):
    """A cloth dropped on a disc made of a fan of thin triangles (apex angle 360/n_fan
    degrees, so every fan triangle meets the centre cell) plus a ring of wide ones."""
    rng = np.random.default_rng(31)
    half = 0.5 * spacing * (n - 1)
    cloth = W.make_cloth(n, n, spacing, (-half, drop, -half), W.K_STRUCT, W.K_SHEAR, W.K_BEND,
                         W.DAMPING, W.NODE_MASS, pins=[], rng=rng)
    th = 2 * np.pi * np.arange(n_fan) / n_fan
    rim = np.stack([0.08 * np.cos(th), np.zeros(n_fan), 0.08 * np.sin(th)], 1)
    out = np.stack([0.16 * np.cos(th), np.zeros(n_fan) - 0.004, 0.16 * np.sin(th)], 1)
    verts = np.concatenate([[[0.0, 0.0, 0.0]], rim, out]).astype(np.float32)
    tris = []
    for k in range(n_fan):
        k1 = (k + 1) % n_fan
        tris.append((0, 1 + k1, 1 + k))  # normal +y
        tris.append((1 + k, 1 + k1, 1 + n_fan + k))
        tris.append((1 + k1, 1 + n_fan + k1, 1 + n_fan + k))
    tris = np.asarray(tris, dtype=np.int32)
    return W._inputs(cloth, verts, tris, thickness=0.005,
                     cell_size=W._surface_cell(verts, tris), dt=1.0 / 600.0, n_substeps=4,
                     n_steps=110, name="cloth on a sliver fan")


def test_sliver_triangles_listed_and_unlisted_queries_agree():
    """On a surface of sliver triangles (closest points on long edges, a crowded centre cell
    that overflows the hit list, nodes with more contacts than a lane of the lanes kernels
    keeps) the listed query, the unlisted one, a 64-slot list and the two- and four-lane
    kernels give the same bits, and one substep matches the oracle."""
    inp = _sliver_fan_scene()
    outs = []
    for cfg in (dict(), dict(hit_slots=0), dict(hit_slots=64, block_threads=256),
                dict(kernel=B.CLOTH_KERNEL_LANES4, hit_slots=8, block_threads=64),
                dict(kernel=B.CLOTH_KERNEL_LANES2, hit_slots=2, block_threads=128),
                dict(kernel=B.CLOTH_KERNEL_LANES4, hit_slots=0, block_threads=64),
                dict(kernel=B.CLOTH_KERNEL_GRID, hit_slots=64, block_threads=64),
                dict(kernel=B.CLOTH_KERNEL_GRID, hit_slots=2, block_threads=64),
                dict(kernel=B.CLOTH_KERNEL_GRID, hit_slots=64, block_threads=128),
                dict(kernel=B.CLOTH_KERNEL_GRID, hit_slots=2, block_threads=128)):
        with B.Cloth(inp) as sim:
            if cfg:
                sim.set_launch(**cfg)
            sim.step(n_steps=inp.n_steps)
            outs.append(sim.read_state())
    for x, v in outs[1:]:
        assert np.array_equal(x, outs[0][0]) and np.array_equal(v, outs[0][1])
    model = oracle.Model.from_inputs(inp)
    with B.Cloth(inp) as sim:
        sim.step(n_steps=inp.n_steps)
        x, v = sim.read_state()
        sim.step(dt=h32(inp), n_substeps=1, n_steps=1)
        x1, v1 = sim.read_state()
    r = one_substep_check(inp, x, v, x1, v1, model, tag="sliver fan")
    assert r["contacts"] > 50


def test_no_collision_defaults_match_direct():
    """Without a surface a grid cloth defaults to the stencil kernel and any other spring
    graph to the tile kernel; both give the one-thread kernel's bits."""
    inp = W.config0(n=48, n_steps=20)
    off = dataclasses.replace(inp, ends=np.concatenate([inp.ends, [[0, 47]]]).astype(np.int32),
                              rest=np.append(inp.rest, np.float32(0.47)),
                              k=np.append(inp.k, np.float32(1.0)),
                              c=np.append(inp.c, np.float32(0.0)))
    for scene, default in ((inp, B.CLOTH_KERNEL_GRID), (off, B.CLOTH_KERNEL_TILE)):
        outs = []
        for cfg in (None, dict(kernel=B.CLOTH_KERNEL_DIRECT, block_threads=64)):
            with B.Cloth(scene) as sim:
                if cfg is None:
                    assert sim.get_launch()["kernel"] == default
                else:
                    sim.set_launch(**cfg)
                sim.step(n_steps=scene.n_steps)
                outs.append(sim.read_state())
        assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_query_volume_counts_match_the_fp32_brute_force():
    """cloth_debug_query_volume on nodes whose prediction is their position (no springs, no
    gravity, at rest): the box hits over all nodes are exactly the FP32 brute-force
    candidate pairs, the distinct candidate triangles those pairs name, and the cell counts
    are consistent (each queried cell counted once, every hit inside a queried cell)."""
    base = W.small_collision_scene(n=24, freq=6)
    rng = np.random.default_rng(77)
    V = base.verts.astype(np.float64)
    P = (V[rng.integers(0, V.shape[0], base.n_nodes)] +
         rng.normal(0, 0.006, size=(base.n_nodes, 3))).astype(np.float32)
    pinned = np.zeros(base.n_nodes, dtype=np.uint8)
    pinned[::17] = 1  # pinned nodes never query
    empty_i = np.zeros((0, 2), dtype=np.int32)
    empty_f = np.zeros(0, dtype=np.float32)
    inp = dataclasses.replace(base, x0=P, v0=np.zeros_like(P), pinned=pinned, ends=empty_i,
                              rest=empty_f, k=empty_f, c=empty_f,
                              kind=np.zeros(0, dtype=np.int8), gravity=(0.0, 0.0, 0.0))
    free = pinned == 0
    pairs = oracle.candidates_f32(P, inp.verts, inp.tris, inp.thickness)
    pairs = pairs[free[pairs[:, 0]]]
    with B.Cloth(inp) as sim:
        for slots in (32, 0):
            sim.set_launch(hit_slots=slots)
            vol = sim.query_volume()
            assert vol["box_hits"] == pairs.shape[0], (slots, vol)
            assert vol["candidate_tris"] == np.unique(pairs[:, 1]).size, (slots, vol)
            assert vol["node_queries"] >= np.unique(pairs[:, 0]).size
            assert vol["node_queries"] <= int(free.sum())
            assert 0 < vol["cells"] <= vol["node_queries"]
            assert vol["cell_refs"] <= vol["refs_tested"] and vol["box_hits"] <= vol["refs_tested"]
    print(f"{pairs.shape[0]} pairs, volume {vol}")
