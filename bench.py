#!/usr/bin/env python3
"""Throughput of the cloth hot path on one MI355X.

One step = one frame of the 316x316-node cloth (99,856 nodes) against the 100,820-triangle
displaced sphere: 4 substeps of spring forces -> integration -> grid broad phase ->
point-triangle narrow phase and response.  Inputs are seeded synthetic data shaped like the
paper's Sec. 4.2 workload, resident in HBM before timing starts.

Prints one JSON line: node-updates/s (one node advanced by one substep), the roofline of the
dominant kernel from HIP events on the library's stream, and the FP64 oracle timed on the
host cores on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300, help="timed frames")
    ap.add_argument("--warmup", type=int, default=20, help="untimed frames")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration)")
    ap.add_argument("--launch", default="",
                    help="launch configuration, e.g. kernel=tile,tile=256,K=4,block=256,graph=1")
    ap.add_argument("--sweep", action="store_true",
                    help="time several launch configurations on the draped state and exit")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched comparison")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint comparison")
    ap.add_argument("--batch-cloths", type=int, default=512)
    ap.add_argument("--no-normals", action="store_true", help="skip the vertex-normal timing")
    ap.add_argument("--no-moving", action="store_true",
                    help="skip the moving-surface / pulled-cloth timing")
    ap.add_argument("--no-mt", action="store_true",
                    help="skip the triangle-triangle narrow-phase timing")
    ap.add_argument("--no-forces-ab", action="store_true",
                    help="skip the gather / scatter force-accumulation comparison")
    return ap.parse_args()


def bench_batched(n_cloths: int, frames: int):
    """512 cloths of side U{16..128}, each over its own 5,120-triangle sphere: one batch handle
    (autotuned launch configuration) against plain per-cloth handles stepped one after another,
    both on this GPU.  Returns node-updates/s of each and the final-state bit identity."""
    import torch

    from paper_2507_11794_amd import cloth, workloads

    cl = workloads.config3(n_cloths=n_cloths)
    n_nodes = sum(c.n_nodes for c in cl)
    sub = cl[0].n_substeps
    stream = torch.cuda.current_stream()
    # one grid cell of one mean surface edge for every cloth (the spheres share their mesh
    # size; 3.5 % faster than the default of two edges, the same contacts)
    cell = float(np.float32(workloads.mean_edge_length(cl[0].verts, cl[0].tris)))
    b = cloth.ClothBatch(cl, stream=stream.cuda_stream, cell_size=cell)
    # the cloths land on their spheres after about 80 frames: tune there, on contacts, as
    # the timed frames run (the tuner restores the state it starts from)
    warm = 100
    b.step(n_steps=warm)
    tuned = b.autotune(frames=4)
    b.step(n_steps=2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(n_steps=frames)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    xb = [b.read_state(i)[0] for i in (0, n_cloths // 2, n_cloths - 1)]
    b.close()
    sims = [cloth.Cloth(dataclasses.replace(c, cell_size=cell), stream=stream.cuda_stream)
            for c in cl]
    for s_ in sims:
        s_.step(n_steps=warm + 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s_ in sims:
        s_.step(n_steps=frames)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    same = all(np.array_equal(sims[i].read_state()[0], x)
               for i, x in zip((0, n_cloths // 2, n_cloths - 1), xb))
    for s_ in sims:
        s_.close()
    upd = n_nodes * sub * frames
    return {"cloths": n_cloths, "nodes": n_nodes, "frames": frames, "first_timed_frame": warm + 2,
            "cell_size": cell,
            "batched_node_updates_per_s": upd / t_batch,
            "plain_per_cloth_node_updates_per_s": upd / t_plain,
            "speedup": t_plain / t_batch, "launch": tuned,
            "bit_identical_sampled_cloths": bool(same)}


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
    sim.step(n_steps=frames)
    # plain stepping of the same frames, timed after a warm-up pass (graph capture) from the
    # initial state
    sim2 = cloth.Cloth(inp, stream=stream.cuda_stream)
    sim2.step(n_steps=frames)
    sim2.write_state(inp.x0, inp.v0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim2.step(n_steps=frames)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    k = torch.tensor(inp.k, device=dev, requires_grad=True)
    c = torch.tensor(inp.c, device=dev, requires_grad=True)
    v0 = torch.zeros((inp.n_nodes, 3), device=dev, requires_grad=True)
    target = torch.zeros((inp.n_nodes, 3), device=dev)
    for rep in range(2):  # the first pass allocates the checkpoint buffers
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x = ClothRollout.apply(sim, k, c, v0, inp.dt, inp.n_substeps, frames, 20, [frames])
        loss = ((x[0] - target) ** 2).sum(dim=1).mean()
        loss.backward()
        torch.cuda.synchronize()
        t_grad = time.perf_counter() - t0
        k.grad = c.grad = v0.grad = None
    sim.close()
    sim2.close()
    upd = inp.n_nodes * inp.n_substeps * frames
    return {"nodes": inp.n_nodes, "frames": frames, "checkpoint_frames": 20,
            "plain_forward_node_updates_per_s": upd / t_plain,
            "forward_backward_node_updates_per_s": upd / t_grad,
            "gradient_cost_vs_plain": t_grad / t_plain}


def bench_normals(sim, n_nodes: int, reps: int = 200):
    """Per-vertex normals of the current state: average kernel time over reps calls, timed
    with HIP events on the handle's stream, against 24 B/node (state read, normal written)."""
    import torch

    stream = torch.cuda.current_stream()
    out = sim.vertex_normals()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(reps):
        sim.vertex_normals(out)
    ev1.record(stream)
    torch.cuda.synchronize()
    us = ev0.elapsed_time(ev1) * 1e3 / reps
    gbs = 24.0 * n_nodes / (us * 1e-6) / 1e9
    return {"nodes": n_nodes, "us_per_call": us, "algorithmic_bytes_per_call": 24 * n_nodes,
            "achieved_gbs": gbs, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS}


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
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    sim.step(n_steps=frames)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    sim.close()
    return {"frames": frames, "nodes": inp.n_nodes, "tris": inp.n_tris,
            "us_per_substep": ms * 1e3 / (frames * inp.n_substeps),
            "node_updates_per_s": inp.n_nodes * inp.n_substeps * frames / (ms * 1e-3)}


FORCES_AB = ["kernel=direct", "kernel=tile,tile=256,K=1,block=256", "kernel=tile,tile=256,K=4,block=256",
             "kernel=scatter_f32", "kernel=scatter_fix"]


def bench_forces_ab(frames: int = 40):
    """Force accumulation compared on the 800x800 hanging cloth (640,000 nodes, 3.83M
    springs, no collision, so the spring pass dominates): the node-centric gather (one
    launch per substep, and temporally blocked tiles) against Alg. 1's spring-centric scatter
    with FP32 atomics and with int32 fixed-point atomics.  Microseconds per substep from HIP
    events over the same frames from the same state."""
    import torch

    from paper_2507_11794_amd import cloth, workloads

    inp = workloads.config2()
    stream = torch.cuda.current_stream()
    sim = cloth.Cloth(inp, stream=stream.cuda_stream)
    sim.step(n_steps=10)
    x0, v0 = sim.read_state()
    out = {"nodes": inp.n_nodes, "springs": inp.n_springs, "frames": frames,
           "substeps_per_frame": inp.n_substeps}
    for text in FORCES_AB:
        sim.set_launch(**{**cloth.launch_dict(cloth.make_launch()), **parse_launch(text)})
        sim.write_state(x0, v0)
        sim.step(n_steps=2)
        sim.write_state(x0, v0)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        sim.step(n_steps=frames)
        ev1.record(stream)
        torch.cuda.synchronize()
        out[text.replace("kernel=", "")] = round(ev0.elapsed_time(ev1) * 1e3 /
                                                 (frames * inp.n_substeps), 3)
    sim.close()
    return out


def parse_launch(text: str) -> dict:
    from paper_2507_11794_amd import cloth

    cfg = {}
    names = {"tile": "tile_nodes", "K": "substeps_per_launch", "block": "block_threads",
             "graph": "use_graph", "hits": "hit_slots", "xcd": "xcd_runs", "split": "split_refs", "sched": "schedule", "wg": "workgroups"}
    for part in filter(None, text.split(",")):
        k, v = part.split("=")
        if k == "kernel":
            cfg["kernel"] = {"tile": cloth.CLOTH_KERNEL_TILE, "direct": cloth.CLOTH_KERNEL_DIRECT,
                             "scatter_f32": cloth.CLOTH_KERNEL_SCATTER_F32,
                             "scatter_fix": cloth.CLOTH_KERNEL_SCATTER_FIX}[v]
        else:
            cfg[names.get(k, k)] = int(v)
    return cfg


SWEEP = [
    "kernel=direct", "kernel=direct,xcd=1", "kernel=direct,xcd=2", "kernel=direct,xcd=4",
    "kernel=direct,xcd=8", "kernel=direct,xcd=16", "kernel=direct,xcd=32", "kernel=direct,xcd=64",
    "kernel=direct,block=128,xcd=8", "kernel=direct,block=256,xcd=4", "kernel=direct,split=48",
    "kernel=direct,hits=48", "kernel=direct,hits=0",
    "kernel=tile,tile=128,K=1,block=256", "kernel=tile,tile=256,K=1,block=256",
    "kernel=scatter_f32", "kernel=scatter_fix",
]


def sweep(inp, frames: int = 40):
    """Time launch configurations from the same draped state (results are bit-identical)."""
    import torch

    from paper_2507_11794_amd import cloth

    stream = torch.cuda.current_stream()
    sim = cloth.Cloth(inp, stream=stream.cuda_stream)
    sim.step(n_steps=150)
    x0, v0 = sim.read_state()
    ref = None
    for text in SWEEP:
        sim.write_state(x0, v0)
        try:
            # every entry starts from the library's defaults, not from the previous entry
            sim.set_launch(**{**cloth.launch_dict(cloth.make_launch()), **parse_launch(text)})
        except cloth.ClothError as e:
            print(json.dumps({"sweep": text, "error": str(e)}), flush=True)
            continue
        sim.step(n_steps=5)
        sim.write_state(x0, v0)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        sim.step(n_steps=frames)
        ev1.record(stream)
        torch.cuda.synchronize()
        us = ev0.elapsed_time(ev1) * 1e3 / (frames * inp.n_substeps)
        x, _ = sim.read_state()
        same = None if ref is None else bool(np.array_equal(x, ref))
        ref = x if ref is None else ref
        print(json.dumps({"sweep": text, "us_per_substep": round(us, 3),
                          "node_updates_per_s": inp.n_nodes / (us * 1e-6),
                          "bit_identical_to_first": same}), flush=True)
    sim.close()
    return 0


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


def counter_traffic(launch: dict):
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE counter summary, if it
    was taken on these kernel sources with this launch configuration; else None."""
    path = os.path.join(ROOT, "profiles", "k_substep_traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("sources_sha256") != sources_sha256():
        return None
    if any(launch.get(k) != v for k, v in rec.get("launch", {}).items()):
        return None
    return rec.get("traffic_bytes_per_launch")


def algorithmic_bytes_per_substep(n_nodes: int, n_springs: int) -> float:
    """Bytes one substep must move: x, v read and written (48 B/node), inverse mass
    (4 B/node), and per spring two end indices plus k, c, rest length (20 B)."""
    return 52.0 * n_nodes + 20.0 * n_springs


def cpu_baseline(inp, x, v, seconds: float):
    import oracle

    model = oracle.Model.from_inputs(inp)
    h = float(np.float32(np.float32(inp.dt) / np.float32(inp.n_substeps)))
    xs, vs = x.astype(np.float64), v.astype(np.float64)
    n_sub = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds and n_sub < 4 * inp.n_steps:
        xs, vs = model.run(xs, vs, h, inp.n_substeps)
        n_sub += inp.n_substeps
    dt = time.perf_counter() - t0
    return {
        "value": inp.n_nodes * n_sub / dt,
        "unit": "node-updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{n_sub} substeps ({n_sub // inp.n_substeps} frames) of the same "
                  f"{inp.n_nodes}-node cloth vs {inp.n_tris}-triangle surface, from the GPU "
                  f"state after the timed frames; single-threaded FP64 C oracle, {dt:.1f} s",
    }


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
    inp = workloads.config1()
    if args.sweep:
        return sweep(inp)
    stream = torch.cuda.current_stream()
    sim = cloth.Cloth(inp, stream=stream.cuda_stream)
    if args.launch:
        sim.set_launch(**parse_launch(args.launch))
    launch = sim.get_launch()
    K = launch["substeps_per_launch"] if launch["kernel"] == cloth.CLOTH_KERNEL_TILE else 1
    sim.step(n_steps=args.warmup)
    torch.cuda.synchronize()

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    sim.step(n_steps=args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    gpu_ms = ev0.elapsed_time(ev1)
    launches = args.steps * inp.n_substeps / K
    kernel_s = gpu_ms * 1e-3 / launches
    node_updates = inp.n_nodes * inp.n_substeps * args.steps
    value = node_updates / wall
    bps = algorithmic_bytes_per_substep(inp.n_nodes, inp.n_springs) * K
    achieved = bps / kernel_s / 1e9
    x, v = sim.read_state()
    info = sim.info()
    normals = None if args.no_normals else bench_normals(sim, inp.n_nodes)
    sim.close()
    out = {
        "metric": "node-updates/s w/ collision, 100K nodes vs 100K tris; batched+adjoint vs plain",
        "value": value,
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
            "grid_cells": info["cells"],
            "grid_refs": info["refs"],
        },
        "roofline": {
            "kernel": ("k_tile (K substeps of fused forces, integration, broad and narrow "
                       "phase per launch)" if K > 1 or launch["kernel"] == cloth.CLOTH_KERNEL_TILE
                       else "k_substep (fused forces, integration, broad and narrow phase)"),
            "launch": launch,
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": counter_traffic(launch),
            "bytes_per_launch": bps,
            "avg_launch_us": kernel_s * 1e6,
        },
    }
    if normals:
        out["normals"] = normals
    if not args.no_moving:
        out["moving_surface"] = bench_moving()
    if not args.no_mt:
        out["mt_narrow_phase"] = bench_mt()
    if not args.no_forces_ab:
        out["forces_ab_us_per_substep"] = bench_forces_ab()
    if not args.no_batch:
        out["batched"] = bench_batched(args.batch_cloths, 200)
    if not args.no_adjoint:
        out["adjoint"] = bench_adjoint(200)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(inp, x, v, args.cpu_seconds)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
