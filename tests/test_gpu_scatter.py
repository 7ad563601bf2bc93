"""GPU spring-centric force accumulation (Alg. 1's scatter form: FP32 atomics and the
WGSL-style int32 fixed point) against the FP64 oracle, plus determinism of the fixed-point
form and its overflow report.  Tolerances as in the other one-substep parity tests; the
fixed point adds at most 2^-25 N per spring (~4e-7 m/s per substep at 1 g, h = 1/2400 s)."""
import numpy as np
import pytest

import oracle
from oracle.parity import substep_parity
from paper_2507_11794_amd import cloth as B
from paper_2507_11794_amd import workloads as W

pytestmark = pytest.mark.gpu

SCATTER = [B.CLOTH_KERNEL_SCATTER_F32, B.CLOTH_KERNEL_SCATTER_FIX]


def h32(inp):
    return float(np.float32(np.float32(inp.dt) / np.float32(inp.n_substeps)))


def side(inp):
    return float(np.max(np.ptp(inp.x0.astype(np.float64), axis=0)))


@pytest.mark.parametrize("kernel", SCATTER)
def test_scatter_one_substep_parity_with_collision(kernel):
    inp = W.small_collision_scene(n=24, n_steps=120)
    model = oracle.Model.from_inputs(inp)
    h = h32(inp)
    contacts = 0
    with B.Cloth(inp) as sim:
        sim.set_launch(kernel=kernel)
        for frame in range(inp.n_steps):
            if frame % 4 == 0 or frame > 70:
                x, v = sim.read_state()
                sim.step(dt=h, n_substeps=1, n_steps=1)
                x1, v1 = sim.read_state()
                r = substep_parity(model, x, v, h, x1, v1, side(inp), tag=f"substep {frame}")
                contacts += r["contacts"]
                sim.step(dt=h, n_substeps=1, n_steps=inp.n_substeps - 1)
            else:
                sim.step(n_steps=1)
    assert contacts > 500


@pytest.mark.parametrize("kernel", SCATTER)
def test_scatter_full_size_parity_hanging_800(kernel):
    inp = W.config2()
    model = oracle.Model.from_inputs(inp)
    h = h32(inp)
    with B.Cloth(inp) as sim:
        sim.set_launch(kernel=kernel)
        sim.step(n_steps=20)
        x, v = sim.read_state()
        sim.step(dt=h, n_substeps=1, n_steps=1)
        x1, v1 = sim.read_state()
    substep_parity(model, x, v, h, x1, v1, side(inp), tag="config2")


def test_fixed_point_is_deterministic_and_float_atomics_close():
    inp = W.small_collision_scene(n=24, n_steps=60)
    runs = []
    for kernel in (B.CLOTH_KERNEL_SCATTER_FIX, B.CLOTH_KERNEL_SCATTER_FIX,
                   B.CLOTH_KERNEL_SCATTER_F32, B.CLOTH_KERNEL_DIRECT):
        with B.Cloth(inp) as sim:
            sim.set_launch(kernel=kernel)
            sim.step(n_steps=15)
            runs.append(sim.read_state())
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    # before contact the three force forms differ only by rounding
    for x, _ in runs[2:]:
        assert np.abs(x.astype(np.float64) - runs[0][0]).max() <= 2e-6 * side(inp)


def test_scatter_with_graphs_batches_and_forces():
    cl = W.config3(n_cloths=3, seed=8, side_lo=12, side_hi=28, freq=6, n_steps=20)
    rng = np.random.default_rng(2)
    f = rng.normal(0, 1e-3, size=(sum(c.n_nodes for c in cl), 3)).astype(np.float32)
    outs = []
    for graph in (0, 1):
        with B.ClothBatch(cl) as b:
            # graphs, and chunks of 3 workgroups dealt to the XCDs: the same bits
            b.set_launch(kernel=B.CLOTH_KERNEL_SCATTER_FIX, use_graph=graph, xcd_runs=3 * graph)
            b.set_external_force(f)
            b.step(n_steps=20)
            outs.append([b.read_state(i) for i in range(len(cl))])
    for a, c in zip(outs[0], outs[1]):
        assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1])
    # close to the gather path with the same forces
    with B.ClothBatch(cl) as b:
        b.set_external_force(f)
        b.step(n_steps=20)
        ref = [b.read_state(i) for i in range(len(cl))]
    for a, r, c in zip(outs[0], ref, cl):
        assert np.abs(a[0].astype(np.float64) - r[0]).max() <= 1e-4 * side(c)


def test_fixed_point_overflow_is_reported():
    # two free nodes 1 m apart joined by a 1 cm spring of 100 N/m: |f| = 99 N > 8 N
    x0 = np.array([[0, 0, 0], [1, 0, 0]], np.float32)
    inp = W.ClothInputs(nx=2, ny=1, x0=x0, v0=np.zeros_like(x0), mass=np.ones(2, np.float32),
                        pinned=np.zeros(2, np.uint8), ends=np.array([[0, 1]], np.int32),
                        rest=np.array([0.01], np.float32), k=np.array([100.0], np.float32),
                        c=np.array([0.0], np.float32), kind=np.zeros(1, np.int8), verts=np.zeros((0, 3), np.float32),
                        tris=np.zeros((0, 3), np.int32), thickness=0.0, cell_size=0.0,
                        dt=1e-4, n_substeps=1, n_steps=1)
    with B.Cloth(inp) as sim:
        sim.set_launch(kernel=B.CLOTH_KERNEL_SCATTER_FIX)
        sim.step(n_steps=1)
        with pytest.raises(B.ClothError) as ei:
            sim.read_state()
        assert ei.value.status == B.CLOTH_ENAN and "fixed-point" in ei.value.detail


def test_rollout_refuses_scatter_kernels():
    import torch
    inp = W.small_collision_scene(n=8, freq=3)
    dev = torch.device("cuda")
    with B.Cloth(inp) as sim:
        sim.set_launch(kernel=B.CLOTH_KERNEL_SCATTER_F32)
        k = torch.tensor(inp.k, device=dev)
        c = torch.tensor(inp.c, device=dev)
        out = torch.zeros((1, inp.n_nodes, 3), device=dev)
        with pytest.raises(B.ClothError) as ei:
            B.cloth_rollout_forward(sim.h, k.data_ptr(), c.data_ptr(), 0, inp.dt, inp.n_substeps,
                                    4, 2, [4], out.data_ptr())
        assert ei.value.status == B.CLOTH_EINVAL
