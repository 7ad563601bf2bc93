#!/usr/bin/env python3
"""Throughput of the cloth hot path on one MI355X.

One step = one frame of the 316x316-node cloth (99,856 nodes) against the 100,820-triangle
displaced sphere: 4 substeps of spring forces -> integration -> grid broad phase ->
point-triangle narrow phase and response.  Inputs are seeded synthetic data shaped like the
paper's Sec. 4.2 workload, resident in HBM before timing starts.

Timing protocol: the cloth is first advanced, untimed, to the draped state (PREROLL frames:
it has landed on the sphere and is sliding over it), then --warmup more frames; the state
there starts every timed window.  One untimed window captures every graph the window replays;
then REPEATS windows of exactly --steps frames are timed from that same state (wall clock and
HIP events on the library's stream, between two device synchronisations), and the median
window is reported.

Prints one JSON line: node-updates/s (one node advanced by one substep), the roofline of the
dominant kernel (algorithmic bytes of the substep, collision share included, over the
kernel's average duration), the same frames with the state copied to the host after each
frame (the PCIe-inclusive rate; never the headline value), the other workloads' legs with
their own rooflines, and the FP64 oracle timed on the host cores on a bounded sample of the
same window.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import multiprocessing as mp
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PREROLL = 150  # frames before the timed window (the cloth lands after about 40)
REPEATS = 5


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed frames per window")
    ap.add_argument("--warmup", type=int, default=5, help="untimed frames after the pre-roll")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=8.0,
                    help="oracle time per CPU leg (single thread, then all cores)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration)")
    ap.add_argument("--launch", default="",
                    help="launch configuration, e.g. kernel=tile,tile=256,K=4,block=256,graph=1")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched comparison")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint comparison")
    ap.add_argument("--batch-cloths", type=int, default=512)
    ap.add_argument("--no-plain", action="store_true",
                    help="batched leg: skip the plain per-cloth comparison (and its collision "
                         "bytes, counted on the plain handles)")
    ap.add_argument("--no-normals", action="store_true", help="skip the vertex-normal timing")
    ap.add_argument("--no-moving", action="store_true",
                    help="skip the moving-surface / pulled-cloth timing")
    ap.add_argument("--no-mt", action="store_true",
                    help="skip the triangle-triangle narrow-phase timing")
    ap.add_argument("--no-forces-ab", action="store_true",
                    help="skip the 800x800 gather / scatter force-accumulation legs")
    ap.add_argument("--only", choices=["forces", "batch", "adjoint", "moving", "mt"],
                    help="run only this leg and print its JSON object (for profiling it)")
    return ap.parse_args()


# ------------------------------------------------------------------ algorithmic bytes

def algorithmic_bytes_per_substep(n_nodes: int, n_springs: int) -> float:
    """Bytes one substep of forces and integration must move: x, v read and written
    (48 B/node), inverse mass (4 B/node), and per spring two end indices plus k, c, rest
    length (20 B)."""
    return 52.0 * n_nodes + 20.0 * n_springs


def collision_bytes(vol: dict) -> float:
    """Bytes of the surface one substep's collision query touches, each array counted once:
    36 B per distinct candidate triangle (its three vertices), 4 B per reference listed in a
    queried non-empty cell, 8 B per queried non-empty cell (its two cell_start entries)."""
    return 36.0 * vol["candidate_tris"] + 4.0 * vol["cell_refs"] + 8.0 * vol["cells"]


# ------------------------------------------------------------------ timing helpers

def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def time_windows(sim, stream, x0, v0, frames: int, repeats: int):
    """`repeats` windows of `frames` frames, each from the state (x0, v0), after one untimed
    window that captures the graphs they replay.  Returns [(wall_s, gpu_ms)] per window."""
    import torch

    sim.write_state(x0, v0)
    sim.step(n_steps=frames)
    torch.cuda.synchronize()
    out = []
    for _ in range(repeats):
        sim.write_state(x0, v0)
        ev0, ev1 = _events()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(stream)
        sim.step(n_steps=frames)
        ev1.record(stream)
        torch.cuda.synchronize()
        out.append((time.perf_counter() - t0, ev0.elapsed_time(ev1)))
    return out


def median_window(windows):
    """The window of median wall time (its wall seconds and GPU milliseconds)."""
    order = sorted(range(len(windows)), key=lambda r: windows[r][0])
    return windows[order[len(order) // 2]]


KERNEL_NAMES = {0: "k_tile", 1: "k_substep", 4: "k_lanes<2>", 5: "k_lanes<4>", 6: "k_grid"}


def kernel_name(launch: dict) -> str:
    return KERNEL_NAMES.get(launch.get("kernel"), "kernel %d" % launch.get("kernel", -1))


def roofline(kernel: str, bytes_per_launch: float, launch_s: float, launch=None, traffic=None):
    achieved = bytes_per_launch / launch_s / 1e9
    out = {"kernel": kernel, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
           "bytes_per_launch": bytes_per_launch, "avg_launch_us": launch_s * 1e6}
    if launch is not None:
        out["launch"] = launch
    return out


# ------------------------------------------------------------------ legs

def bench_batched(n_cloths: int, frames: int, plain: bool = True):
    """512 cloths of side U{16..128}, each over its own 5,120-triangle sphere: one batch handle
    (autotuned launch configuration) against plain per-cloth handles stepped one after another,
    both on this GPU, over the same frames from the same state (frame 100: every cloth is on
    its sphere).  Returns node-updates/s of each, the batch kernel's roofline (collision share
    counted on the per-cloth handles, whose states are bit-identical) and the final-state bit
    identity of sampled cloths."""
    import torch

    from paper_2507_11794_amd import cloth, workloads

    cl = workloads.config3(n_cloths=n_cloths)
    n_nodes = sum(c.n_nodes for c in cl)
    n_springs = sum(c.n_springs for c in cl)
    sub = cl[0].n_substeps
    stream = torch.cuda.current_stream()
    # one grid cell of one mean surface edge for every cloth (the spheres share their mesh
    # size; 3.5 % faster than the default of two edges, the same contacts)
    cell = float(np.float32(workloads.mean_edge_length(cl[0].verts, cl[0].tris)))
    b = cloth.ClothBatch(cl, stream=stream.cuda_stream, cell_size=cell)
    warm = 100
    b.step(n_steps=warm)
    # tune on contacts, as the timed frames run (the tuner restores the state it starts from)
    tuned = b.autotune(frames=16)
    b.step(n_steps=frames)  # untimed: captures the graphs of a window of this length
    torch.cuda.synchronize()
    b.step(n_steps=2)
    torch.cuda.synchronize()
    ev0, ev1 = _events()
    t0 = time.perf_counter()
    ev0.record(stream)
    b.step(n_steps=frames)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    first = warm + frames + 2
    sample = (0, n_cloths // 2, n_cloths - 1)
    xb = [b.read_state(i)[0] for i in sample]
    b.close()
    upd = n_nodes * sub * frames
    K = tuned.get("substeps_per_launch", 1) if tuned.get("kernel") == cloth.CLOTH_KERNEL_TILE else 1
    launch_s = gpu_ms * 1e-3 / (frames * sub / K)
    if not plain:
        return {"cloths": n_cloths, "nodes": n_nodes, "springs": n_springs, "frames": frames,
                "first_timed_frame": first, "cell_size": cell,
                "batched_node_updates_per_s": upd / t_batch, "launch": tuned,
                "avg_launch_us": launch_s * 1e6}
    sims = [cloth.Cloth(dataclasses.replace(c, cell_size=cell), stream=stream.cuda_stream)
            for c in cl]
    for s_ in sims:
        s_.step(n_steps=first)
    torch.cuda.synchronize()
    coll = sum(collision_bytes(s_.query_volume()) for s_ in sims)
    t0 = time.perf_counter()
    for s_ in sims:
        s_.step(n_steps=frames)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    same = all(np.array_equal(sims[i].read_state()[0], x) for i, x in zip(sample, xb))
    for s_ in sims:
        s_.close()
    per_sub = algorithmic_bytes_per_substep(n_nodes, n_springs) + coll
    return {"cloths": n_cloths, "nodes": n_nodes, "springs": n_springs, "frames": frames,
            "first_timed_frame": first, "cell_size": cell,
            "batched_node_updates_per_s": upd / t_batch,
            "plain_per_cloth_node_updates_per_s": upd / t_plain,
            "speedup": t_plain / t_batch, "launch": tuned,
            "collision_bytes_per_substep": coll,
            "roofline": roofline(f"{kernel_name(tuned)} (512 cloths, autotuned launch)",
                                 per_sub * K, launch_s, tuned,
                                 counter_traffic(tuned, "batch512")),
            "bit_identical_sampled_cloths": bool(same)}


def adjoint_bytes_per_substep(n_nodes: int, n_springs: int, coll: float) -> float:
    """Bytes one substep of the gradient run moves, each array counted once per pass: the
    forward substep (52 B/node + 20 B/spring + collision), its recompute from the checkpoint
    (the same, plus the stored prediction, 12 B/node), and the backward substep: the node
    pass reads the state, prediction, inverse mass and output adjoints (64 B/node) and writes
    the partial adjoints and the force adjoint (36 B/node), the spring pass reads the state,
    force and partial adjoints (60 B/node) and writes the input adjoints (24 B/node), per
    spring the ends and parameters (20 B) and dL/dk, dL/dc in FP64, read and written
    (32 B), plus the collision query again."""
    fwd = algorithmic_bytes_per_substep(n_nodes, n_springs) + coll
    rec = fwd + 12.0 * n_nodes
    bwd = (64.0 + 36.0 + 60.0 + 24.0) * n_nodes + (20.0 + 32.0) * n_springs + coll
    return fwd + rec + bwd


def bench_adjoint(frames: int = 200):
    """64x64 cloth over a 2,000-triangle sphere, trajectory loss on the final frame, gradients
    for per-spring k, c and v0 with checkpoints every 20 frames: forward + recompute + backward
    against plain forward stepping of the same frames on this GPU."""
    import torch

    from paper_2507_11794_amd import cloth, workloads
    from paper_2507_11794_amd.rollout import ClothRollout

    inp, k_hat = workloads.config4(n_steps=frames)
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream()
    sim = cloth.Cloth(inp, stream=stream.cuda_stream)
    sim2 = cloth.Cloth(inp, stream=stream.cuda_stream)
    fwd_kernel = kernel_name(sim2.get_launch())
    sim2.step(n_steps=frames)  # untimed: graph capture
    sim2.write_state(inp.x0, inp.v0)
    sim2.step(n_steps=frames // 2)
    coll = collision_bytes(sim2.query_volume())  # mid-run (the cloth is on the sphere)
    sim2.write_state(inp.x0, inp.v0)
    torch.cuda.synchronize()
    ev0, ev1 = _events()
    t0 = time.perf_counter()
    ev0.record(stream)
    sim2.step(n_steps=frames)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    plain_ms = ev0.elapsed_time(ev1)
    k = torch.tensor(inp.k, device=dev, requires_grad=True)
    c = torch.tensor(inp.c, device=dev, requires_grad=True)
    v0 = torch.zeros((inp.n_nodes, 3), device=dev, requires_grad=True)
    target = torch.zeros((inp.n_nodes, 3), device=dev)
    times = []
    for rep in range(3):  # the first pass allocates the checkpoint buffers
        torch.cuda.synchronize()
        ev0, ev1 = _events()
        t0 = time.perf_counter()
        ev0.record(stream)
        x = ClothRollout.apply(sim, k, c, v0, inp.dt, inp.n_substeps, frames, 20, [frames])
        loss = ((x[0] - target) ** 2).sum(dim=1).mean()
        loss.backward()
        ev1.record(stream)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0, ev0.elapsed_time(ev1)))
        k.grad = c.grad = v0.grad = None
    sim.close()
    sim2.close()
    t_grad, grad_ms = median_window(times[1:])
    n_sub = inp.n_substeps * frames
    upd = inp.n_nodes * n_sub
    per_sub = adjoint_bytes_per_substep(inp.n_nodes, inp.n_springs, coll)
    return {"nodes": inp.n_nodes, "frames": frames, "checkpoint_frames": 20,
            "plain_forward_node_updates_per_s": upd / t_plain,
            "forward_backward_node_updates_per_s": upd / t_grad,
            "gradient_cost_vs_plain": t_grad / t_plain,
            "plain_forward_roofline": roofline(
                f"{fwd_kernel} (64x64 cloth: 64 wavefronts, latency-bound)",
                algorithmic_bytes_per_substep(inp.n_nodes, inp.n_springs) + coll,
                plain_ms * 1e-3 / n_sub),
            "gradient_roofline": roofline(
                "forward + recompute + adjoint kernels, per substep", per_sub,
                grad_ms * 1e-3 / n_sub)}


def bench_normals(sim, n_nodes: int, reps: int = 200):
    """Per-vertex normals of the current state: average kernel time over reps calls, timed
    with HIP events on the handle's stream, against 24 B/node (state read, normal written)."""
    import torch

    stream = torch.cuda.current_stream()
    out = sim.vertex_normals()
    torch.cuda.synchronize()
    ev0, ev1 = _events()
    ev0.record(stream)
    for _ in range(reps):
        sim.vertex_normals(out)
    ev1.record(stream)
    torch.cuda.synchronize()
    us = ev0.elapsed_time(ev1) * 1e3 / reps
    gbs = 24.0 * n_nodes / (us * 1e-6) / 1e9
    return {"nodes": n_nodes, "us_per_call": us, "algorithmic_bytes_per_call": 24 * n_nodes,
            "achieved_gbs": gbs, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS}


def bench_read_back(sim, x0, v0, n_nodes: int, n_substeps: int, frames: int):
    """Stepping with the state copied to the host after every frame (cloth_read_state into
    the same two arrays each time: AoS in node-id order, synchronising), from the state
    (x0, v0): the rate a caller that takes host buffers over the boundary each frame sees,
    PCIe copies included."""
    x = np.empty((n_nodes, 3), dtype=np.float32)
    v = np.empty((n_nodes, 3), dtype=np.float32)
    sim.write_state(x0, v0)
    sim.step(n_steps=1)
    sim.read_state(x, v)
    sim.write_state(x0, v0)
    t0 = time.perf_counter()
    for _ in range(frames):
        sim.step(n_steps=1)
        sim.read_state(x, v)
    wall = time.perf_counter() - t0
    return {"frames": frames, "ms_per_frame": wall * 1e3 / frames,
            "node_updates_per_s": n_nodes * n_substeps * frames / wall,
            "host_bytes_per_frame": 24 * n_nodes}


def coarse_cells(inp):
    """The workload with a broad-phase grid cell of 2 x the mean surface edge."""
    from paper_2507_11794_amd import workloads

    cell = float(np.float32(2.0 * workloads.mean_edge_length(inp.verts, inp.tris)))
    return dataclasses.replace(inp, cell_size=cell)


def bench_moving(frames: int = 60):
    """The 316x316 cloth over the 100,820-triangle sphere while the sphere moves every frame
    (its grid rebuilt on the device before each frame) and the cloth's last row is pulled
    along +x: frame throughput, and the surface update's own cost."""
    import torch

    from paper_2507_11794_amd import cloth, workloads

    # a surface rebuilt every frame: the coarser grid of 2 x the mean edge has a quarter of
    # the references to rebuild
    inp = coarse_cells(workloads.config1())
    n = inp.nx
    f = np.zeros((inp.n_nodes, 3), dtype=np.float32)
    f[(n - 1) * n:, 0] = 0.002
    stream = torch.cuda.current_stream()
    sim = cloth.Cloth(inp, stream=stream.cuda_stream)
    sim.set_external_force(f)
    sim.step(n_steps=100)
    verts = [workloads.moving_surface(inp.verts, 100 + i, inp.dt) for i in range(frames)]
    torch.cuda.synchronize()
    t_upd = 0.0
    t0 = time.perf_counter()
    for V in verts:
        ta = time.perf_counter()
        sim.update_surface(V)
        t_upd += time.perf_counter() - ta
        sim.step(n_steps=1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    info = sim.info()
    sim.close()
    return {"frames": frames, "nodes": inp.n_nodes, "tris": inp.n_tris, "grid_refs": info["refs"],
            "node_updates_per_s": inp.n_nodes * inp.n_substeps * frames / wall,
            "ms_per_frame": wall * 1e3 / frames,
            "surface_update_ms": t_upd * 1e3 / frames}


def bench_mt(frames: int = 30):
    """The benchmark workload with the triangle-triangle narrow phase (extended
    Moller-Trumbore): frames timed after the drop (110 frames in), node-updates/s."""
    import torch

    from paper_2507_11794_amd import cloth, workloads

    # the swept query visits every cell under a node's path and edges: coarser cells
    # (2 x the mean edge) suit it better than the proximity query's one-edge cells
    inp = coarse_cells(workloads.config1())
    stream = torch.cuda.current_stream()
    sim = cloth.Cloth(inp, flags=cloth.CLOTH_F_NARROW_MT, stream=stream.cuda_stream)
    sim.step(n_steps=110)
    x0, v0 = sim.read_state()
    wall, ms = median_window(time_windows(sim, stream, x0, v0, frames, 3))
    sim.close()
    return {"frames": frames, "first_timed_frame": 110, "nodes": inp.n_nodes, "tris": inp.n_tris,
            "us_per_substep": ms * 1e3 / (frames * inp.n_substeps),
            "node_updates_per_s": inp.n_nodes * inp.n_substeps * frames / wall}


FORCES_AB = ["kernel=direct", "kernel=grid", "kernel=grid,xcd=16", "kernel=tile,tile=256,K=1,block=256",
             "kernel=tile,tile=256,K=4,block=256", "kernel=scatter_f32", "kernel=scatter_fix"]


def bench_forces_ab(frames: int = 40):
    """The 800x800 hanging cloth (640,000 nodes, 3.83M springs, no collision, so the spring
    pass dominates): the node-centric gathers (one thread per node from the incidence lists;
    the grid-stencil kernel, in the hardware's workgroup order and in chunks of 16 tiles per
    XCD, its default; temporally blocked tiles) against Alg. 1's spring-centric scatter with
    FP32 atomics and with int32 fixed-point atomics.  Microseconds per substep from HIP
    events (median of 3 windows from the same state, graphs captured beforehand), and the
    roofline of the default launch."""
    import torch

    from paper_2507_11794_amd import cloth, workloads

    inp = workloads.config2()
    stream = torch.cuda.current_stream()
    sim = cloth.Cloth(inp, stream=stream.cuda_stream)
    default = sim.get_launch()
    sim.step(n_steps=10)
    x0, v0 = sim.read_state()
    out = {"nodes": inp.n_nodes, "springs": inp.n_springs, "frames": frames,
           "substeps_per_frame": inp.n_substeps}
    for text in FORCES_AB:
        sim.set_launch(**{**cloth.launch_dict(cloth.make_launch()), **parse_launch(text)})
        _, ms = median_window(time_windows(sim, stream, x0, v0, frames, 3))
        out[text.replace("kernel=", "")] = round(ms * 1e3 / (frames * inp.n_substeps), 3)
    sim.set_launch(**default)
    _, ms = median_window(time_windows(sim, stream, x0, v0, frames, 3))
    sim.close()
    K = default["substeps_per_launch"] if default["kernel"] == cloth.CLOTH_KERNEL_TILE else 1
    launch_s = ms * 1e-3 / (frames * inp.n_substeps / K)
    out["roofline"] = roofline(
        f"{kernel_name(default)} (default launch without a surface)",
        algorithmic_bytes_per_substep(inp.n_nodes, inp.n_springs) * K, launch_s, default,
        counter_traffic(default, "cloth800_hanging"))
    return out


def parse_launch(text: str) -> dict:
    from paper_2507_11794_amd import cloth

    cfg = {}
    names = {"tile": "tile_nodes", "K": "substeps_per_launch", "block": "block_threads",
             "graph": "use_graph", "hits": "hit_slots", "xcd": "xcd_runs", "split": "split_refs",
             "sched": "schedule", "wg": "workgroups"}
    for part in filter(None, text.split(",")):
        k, v = part.split("=")
        if k == "kernel":
            cfg["kernel"] = {"tile": cloth.CLOTH_KERNEL_TILE, "direct": cloth.CLOTH_KERNEL_DIRECT,
                             "scatter_f32": cloth.CLOTH_KERNEL_SCATTER_F32,
                             "scatter_fix": cloth.CLOTH_KERNEL_SCATTER_FIX,
                             "lanes2": cloth.CLOTH_KERNEL_LANES2,
                             "lanes4": cloth.CLOTH_KERNEL_LANES4,
                             "grid": cloth.CLOTH_KERNEL_GRID}[v]
        else:
            cfg[names.get(k, k)] = int(v)
    return cfg


def calibrate_copy(mib: int, reps: int = 5):
    """A plain device-to-device copy of known size, for scaling memory counters."""
    import torch

    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes_read": n * 4, "bytes_written": n * 4, "reps": reps}))
    return 0


def sources_sha256() -> str:
    """Hash of the HIP library's sources (file names and contents, sorted)."""
    import glob
    import hashlib

    csrc = os.path.join(ROOT, "paper_2507_11794_amd", "csrc")
    files = sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.h")) +
                   glob.glob(os.path.join(csrc, "*.cpp")))
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()


def counter_traffic(launch: dict, workload: str):
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE counter summary of this
    workload's kernel, if it was taken on these kernel sources with this launch
    configuration; else None."""
    path = os.path.join(ROOT, "profiles", "counter_traffic.json")
    try:
        recs = json.load(open(path))
    except (OSError, ValueError):
        return None
    for rec in recs:
        if rec.get("workload") != workload or rec.get("kernel") != kernel_name(launch):
            continue
        if rec.get("sources_sha256") != sources_sha256():
            continue
        if any(launch.get(k) != v for k, v in rec.get("launch", {}).items()):
            continue
        return rec.get("traffic_bytes_per_launch")
    return None


# ------------------------------------------------------------------ CPU baseline

def _oracle_leg(args):
    """One oracle process: the workload's model, the window's starting state, substeps until
    `seconds` have passed (started together with the other processes at `barrier`).  Returns
    (substeps, seconds, start, end)."""
    x, v, seconds, barrier = args
    import oracle
    from paper_2507_11794_amd import workloads

    inp = workloads.config1()
    model = oracle.Model.from_inputs(inp)
    h = float(np.float32(np.float32(inp.dt) / np.float32(inp.n_substeps)))
    xs, vs = x.astype(np.float64), v.astype(np.float64)
    if barrier is not None:
        barrier.wait()
    n_sub = 0
    t0 = time.perf_counter()
    start = time.time()
    while time.perf_counter() - t0 < seconds:
        xs, vs = model.run(xs, vs, h, 1)
        n_sub += 1
    return n_sub, time.perf_counter() - t0, start, time.time()


def _proc_leg(q, args):
    q.put(_oracle_leg(args))


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(inp, x, v, seconds: float):
    """The FP64 oracle on the host cores from the timed window's starting state: one process
    (single thread), then one process per core of this process's affinity (at most 16, the
    host share of one GPU), each stepping its own copy of the workload, started together.
    The oracle itself is single-threaded."""
    n1, t1, _, _ = _oracle_leg((x, v, seconds, None))
    single = inp.n_nodes * n1 / t1
    cores = len(os.sched_getaffinity(0))
    P = max(1, min(cores, 16))
    ctx = mp.get_context("spawn")
    barrier = ctx.Barrier(P)
    q = ctx.Queue()
    procs = [ctx.Process(target=_proc_leg, args=(q, (x, v, seconds, barrier))) for _ in range(P)]
    for p in procs:
        p.start()
    res = [q.get(timeout=600) for _ in procs]
    for p in procs:
        p.join()
    subs = sum(r[0] for r in res)
    span = max(r[3] for r in res) - min(r[2] for r in res)
    allc = inp.n_nodes * subs / span
    return {
        "value": allc,
        "unit": "node-updates/s",
        "cores": P,
        "kind": "oracle",
        "single_thread_value": single,
        "cpu_model": cpu_model(),
        "affinity_cores": cores,
        "os_cpu_count": os.cpu_count(),
        "sample": f"the {inp.n_nodes}-node cloth vs {inp.n_tris}-triangle surface from the timed "
                  f"window's starting (draped) state: single thread {n1} substeps in {t1:.1f} s; "
                  f"then {P} processes, one per core, each stepping its own copy for "
                  f"{seconds:.0f} s ({subs} substeps in all over {span:.1f} s); single-threaded "
                  f"FP64 C oracle",
    }


# ------------------------------------------------------------------ main

def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "path is a design, not a build", file=sys.stderr)
        return 2
    import torch

    from paper_2507_11794_amd import cloth, workloads

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        return calibrate_copy(args.calibrate_copy)
    if args.only:
        leg = {"forces": bench_forces_ab, "batch": lambda: bench_batched(args.batch_cloths, 200, not args.no_plain),
               "adjoint": lambda: bench_adjoint(200), "moving": bench_moving,
               "mt": bench_mt}[args.only]
        print(json.dumps({args.only: leg()}))
        return 0
    inp = workloads.config1()
    stream = torch.cuda.current_stream()
    sim = cloth.Cloth(inp, stream=stream.cuda_stream)
    if args.launch:
        sim.set_launch(**parse_launch(args.launch))
    launch = sim.get_launch()
    K = launch["substeps_per_launch"] if launch["kernel"] == cloth.CLOTH_KERNEL_TILE else 1
    sim.step(n_steps=PREROLL + args.warmup)
    x0, v0 = sim.read_state()
    vol0 = sim.query_volume()
    windows = time_windows(sim, stream, x0, v0, args.steps, REPEATS)
    vol1 = sim.query_volume()
    wall, gpu_ms = median_window(windows)
    launches = args.steps * inp.n_substeps / K
    kernel_s = gpu_ms * 1e-3 / launches
    node_updates = inp.n_nodes * inp.n_substeps * args.steps
    coll = 0.5 * (collision_bytes(vol0) + collision_bytes(vol1))
    per_sub = algorithmic_bytes_per_substep(inp.n_nodes, inp.n_springs) + coll
    info = sim.info()
    normals = None if args.no_normals else bench_normals(sim, inp.n_nodes)
    read_back = bench_read_back(sim, x0, v0, inp.n_nodes, inp.n_substeps, args.steps)
    sim.close()
    first = PREROLL + args.warmup
    out = {
        "metric": "node-updates/s w/ collision, 100K nodes vs 100K tris; batched+adjoint vs plain",
        "value": node_updates / wall,
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"cloth {inp.nx}x{inp.ny} ({inp.n_nodes} nodes, {inp.n_springs} springs) "
                        f"dropped on a displaced sphere of {inp.n_tris} triangles; "
                        f"{inp.n_substeps} substeps per frame, dt = 1/600 s",
            "substeps_per_step": inp.n_substeps,
            "first_timed_frame": first,
            "timing": f"median of {REPEATS} windows of {args.steps} frames from the state at "
                      f"frame {first} (graphs captured beforehand)",
            "window_wall_s": [round(w[0], 6) for w in windows],
            "grid_cell_m": float(np.float32(inp.cell_size)),
            "grid_cell_note": "one mean surface edge (the library default is two; the contacts "
                              "do not depend on it)",
            "grid_cells": info["cells"],
            "grid_refs": info["refs"],
            "collision_query": {"start": vol0, "end": vol1},
        },
        "roofline": roofline(
            f"{kernel_name(launch)} (K substeps of fused forces, integration, broad and narrow "
            "phase per launch)" if launch["kernel"] == cloth.CLOTH_KERNEL_TILE
            else f"{kernel_name(launch)} (fused forces, integration, broad and narrow phase)",
            per_sub * K, kernel_s, launch, counter_traffic(launch, "cloth316_sphere100k")),
    }
    out["roofline"]["bytes_per_node_update"] = per_sub / inp.n_nodes
    out["roofline"]["collision_bytes_per_substep"] = coll
    out["read_back_each_frame"] = read_back
    if normals:
        out["normals"] = normals
    if not args.no_moving:
        out["moving_surface"] = bench_moving()
    if not args.no_mt:
        out["mt_narrow_phase"] = bench_mt()
    if not args.no_forces_ab:
        out["forces_800x800"] = bench_forces_ab()
    if not args.no_batch:
        out["batched"] = bench_batched(args.batch_cloths, 200)
    if not args.no_adjoint:
        out["adjoint"] = bench_adjoint(200)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(inp, x0, v0, args.cpu_seconds)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
