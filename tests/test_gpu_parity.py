"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same seeded
inputs.

Tolerances.  FP32 rounds positions of ~1 m magnitude to ~6e-8 m; one substep moves a node by
h v* with v* carrying the spring-force rounding (differences of FP32 positions, ~1e-7
relative) divided by the node mass, so one-substep positions agree to a few ulps of the
coordinates (bar: 2e-6 of the cloth side) and velocities to ~1e-4 m/s (bar: 2e-3 m/s plus
1e-4 relative).  Over 100 frames of the collision-free hanging cloth the FP32 trajectory
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
    inp = list(_tiny_surfaces())[which]
    rng = np.random.default_rng(100 + which)
    V = inp.verts.astype(np.float64)
    th = np.float32(inp.thickness)
    pts = [V[rng.integers(0, V.shape[0], 1500)] + rng.normal(0, 0.008, size=(1500, 3))]
    # far outside the grid
    pts.append(rng.uniform(-3, 3, size=(200, 3)))
    # exactly on, and one ulp outside / inside, inflated box faces
    T = inp.tris
    lo = np.min(inp.verts[T], axis=1) - th
    hi = np.max(inp.verts[T], axis=1) + th
    pick = rng.integers(0, T.shape[0], 200)
    for bound in (lo[pick], hi[pick]):
        base = (lo[pick] + hi[pick]) * np.float32(0.5)
        for axis in range(3):
            for d in (-1, 0, 1):
                q = base.copy()
                q[:, axis] = bound[:, axis]
                if d:
                    q[:, axis] = np.nextafter(q[:, axis], np.float32(d * np.inf))
                pts.append(q.astype(np.float64))
    P = np.concatenate(pts).astype(np.float32)
    with B.Cloth(inp) as sim:
        info = sim.info()
        got = sim.debug_candidates(P)
        # also points on grid cell faces of the handle's own grid
        assert info["cells"] > 0
    want = oracle.candidates_f32(P, inp.verts, inp.tris, inp.thickness)
    print(f"surface {which}: {P.shape[0]} points, {want.shape[0]} pairs, grid {info}")
    assert got.shape == want.shape and np.array_equal(got, want)


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


@pytest.mark.parametrize("frames", [0, 60, 150, 299])
def test_config1_full_size_one_substep_parity(frames):
    inp = W.config1()
    model = oracle.Model.from_inputs(inp)
    with B.Cloth(inp) as sim:
        if frames:
            sim.step(n_steps=frames)
        x, v = sim.read_state()
        sim.step(dt=h32(inp), n_substeps=1, n_steps=1)
        x1, v1 = sim.read_state()
    r = one_substep_check(inp, x, v, x1, v1, model, tag=f"config1 frame {frames}")
    print(f"config1 frame {frames}: {r}")
    if frames >= 150:
        assert r["contacts"] > 1000


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


@pytest.mark.parametrize("kernel", [B.CLOTH_KERNEL_DIRECT, B.CLOTH_KERNEL_TILE])
def test_default_and_tile_kernels_match_oracle_one_substep(kernel):
    inp = W.config1(n=96, freq=24)
    model = oracle.Model.from_inputs(inp)
    with B.Cloth(inp) as sim:
        if kernel == B.CLOTH_KERNEL_DIRECT:
            assert sim.get_launch()["kernel"] == B.CLOTH_KERNEL_DIRECT  # the default
        else:
            sim.set_launch(kernel=kernel, block_threads=256)
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
    that overflows the hit list) the listed query, the unlisted one and a 64-slot list give
    the same bits, and one substep matches the oracle."""
    inp = _sliver_fan_scene()
    outs = []
    for cfg in (dict(), dict(hit_slots=0), dict(hit_slots=64, block_threads=256)):
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


def test_no_collision_default_is_the_tile_kernel_and_matches_direct():
    inp = W.config0(n=48, n_steps=20)
    outs = []
    for cfg in (None, dict(kernel=B.CLOTH_KERNEL_DIRECT, block_threads=64)):
        with B.Cloth(inp) as sim:
            if cfg is None:
                assert sim.get_launch()["kernel"] == B.CLOTH_KERNEL_TILE
            else:
                sim.set_launch(**cfg)
            sim.step(n_steps=inp.n_steps)
            outs.append(sim.read_state())
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
