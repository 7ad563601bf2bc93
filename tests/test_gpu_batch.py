"""GPU batched mode: many uneven cloths in one handle evolve exactly (bit for bit) as plain
per-cloth handles do, for every launch configuration and schedule, and after autotuning."""
import dataclasses

import numpy as np
import pytest

import oracle
from oracle.parity import substep_parity
from paper_2507_11794_amd import cloth as B
from paper_2507_11794_amd import workloads as W

pytestmark = pytest.mark.gpu


def _cloths(n=6, seed=77, hi=48):
    return W.config3(n_cloths=n, seed=seed, side_lo=16, side_hi=hi, freq=8, n_steps=30)


def _plain(inp, frames):
    with B.Cloth(inp) as s:
        s.step(n_steps=frames)
        return s.read_state()


def test_batch_equals_plain_per_cloth_bitwise():
    cl = _cloths()
    frames = 30
    with B.ClothBatch(cl) as b:
        info = b.info()
        assert info["cloths"] == len(cl)
        assert info["nodes"] == sum(c.n_nodes for c in cl)
        b.step(n_steps=frames)
        got = [b.read_state(i) for i in range(len(cl))]
    for i, c in enumerate(cl):
        xp, vp = _plain(c, frames)
        assert np.array_equal(got[i][0], xp) and np.array_equal(got[i][1], vp), i
    moved = max(np.abs(g[0] - c.x0).max() for g, c in zip(got, cl))
    assert moved > 0.01


def _with_distinct_k(c, n_distinct, seed):
    """c with its first n_distinct springs given their own stiffness (a table entry each)."""
    k = c.k.copy()
    k[:n_distinct] *= 1.0 + np.random.default_rng(seed).uniform(0.01, 0.05, n_distinct).astype(np.float32)
    return dataclasses.replace(c, k=k)


@pytest.mark.parametrize("case", ["bytes, table in LDS", "bytes, table in memory",
                                  "full entries"])
def test_batch_parameter_tables_per_cloth_equal_plain_handles(case):
    """Each cloth's parameter entries form their own range of the table: with 90 cloths of
    three entries each (270 in all, more than one byte can index) the stencil kernel still
    reads byte entries relative to the cloth's first and stages the cloth's entries in LDS;
    with cloths of 129-255 entries it reads the table from memory; with a cloth of more than
    255 it reads the full entries.  Every cloth ends bit-identical to its own handle."""
    if case == "bytes, table in LDS":
        cl = W.config3(n_cloths=90, seed=31, side_lo=16, side_hi=16, freq=6, n_steps=10)
    else:
        base = W.config3(n_cloths=3, seed=32, side_lo=16, side_hi=20, freq=6, n_steps=10)
        n = [150, 200, 40] if case == "bytes, table in memory" else [150, 400, 40]
        cl = [_with_distinct_k(c, m, 40 + i) for i, (c, m) in enumerate(zip(base, n))]
    frames = 10
    with B.ClothBatch(cl) as b:
        assert b.get_launch()["kernel"] == B.CLOTH_KERNEL_GRID
        assert b.get_launch()["block_threads"] == 64  # one wavefront per tile for batches
        b.step(n_steps=frames)
        got = [b.read_state(i) for i in range(len(cl))]
    for i, c in enumerate(cl):
        xp, vp = _plain(c, frames)
        assert np.array_equal(got[i][0], xp) and np.array_equal(got[i][1], vp), (case, i)


SCHEDULES = [
    dict(kernel=B.CLOTH_KERNEL_DIRECT),
    dict(kernel=B.CLOTH_KERNEL_TILE, tile_nodes=128, substeps_per_launch=2),
    dict(kernel=B.CLOTH_KERNEL_TILE, tile_nodes=256, substeps_per_launch=4,
         schedule=B.CLOTH_SCHED_LPT, workgroups=5),
    dict(kernel=B.CLOTH_KERNEL_TILE, tile_nodes=64, substeps_per_launch=3,
         schedule=B.CLOTH_SCHED_RR, workgroups=7, use_graph=0),
    dict(kernel=B.CLOTH_KERNEL_LANES4, block_threads=64, hit_slots=8),
    dict(kernel=B.CLOTH_KERNEL_LANES2, block_threads=256, hit_slots=4, xcd_runs=2),
    dict(kernel=B.CLOTH_KERNEL_GRID, block_threads=64),
    dict(kernel=B.CLOTH_KERNEL_GRID, block_threads=64, hit_slots=4, xcd_runs=2),
    dict(kernel=B.CLOTH_KERNEL_GRID, block_threads=128),
    dict(kernel=B.CLOTH_KERNEL_GRID, block_threads=128, hit_slots=4, xcd_runs=2),
]


def test_batch_launch_configurations_bit_identical():
    cl = _cloths(n=5, seed=5)
    outs = []
    for cfg in SCHEDULES:
        with B.ClothBatch(cl) as b:
            b.set_launch(**cfg)
            b.step(n_steps=25)
            outs.append([b.read_state(i) for i in range(len(cl))])
    for o in outs[1:]:
        for (x, v), (xr, vr) in zip(o, outs[0]):
            assert np.array_equal(x, xr) and np.array_equal(v, vr)


def test_autotune_picks_a_valid_configuration_without_changing_results():
    cl = _cloths(n=4, seed=9)
    with B.ClothBatch(cl) as b:
        b.step(n_steps=10)
        ref = B.ClothBatch(cl)
        ref.step(n_steps=10)
        best = b.autotune(frames=2)
        assert best["kernel"] in (B.CLOTH_KERNEL_TILE, B.CLOTH_KERNEL_DIRECT,
                                  B.CLOTH_KERNEL_LANES2, B.CLOTH_KERNEL_LANES4,
                                  B.CLOTH_KERNEL_GRID)
        assert b.get_launch() == best
        b.step(n_steps=15)
        ref.step(n_steps=15)
        for i in range(len(cl)):
            x, v = b.read_state(i)
            xr, vr = ref.read_state(i)
            assert np.array_equal(x, xr) and np.array_equal(v, vr)
        ref.close()


def test_batch_cloth_one_substep_parity_with_oracle():
    cl = _cloths(n=3, seed=21)
    h = float(np.float32(np.float32(cl[0].dt) / np.float32(cl[0].n_substeps)))
    with B.ClothBatch(cl) as b:
        b.step(n_steps=40)
        states = [b.read_state(i) for i in range(len(cl))]
        b.step(n_steps=1, dt=h, n_substeps=1)
        nxt = [b.read_state(i) for i in range(len(cl))]
    for i, c in enumerate(cl):
        m = oracle.Model.from_inputs(c)
        L = float(np.max(np.ptp(c.x0.astype(np.float64), axis=0)))
        substep_parity(m, states[i][0], states[i][1], h, nxt[i][0], nxt[i][1], L,
                       tag=f"batch cloth {i}")
