"""Host logic of the benchmark: it refuses more than one GPU, counts the algorithmic bytes of
a substep, parses launch strings, and reports counter traffic only for the kernel sources
and launch configuration the committed counters were taken on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr and r.stdout.strip() == ""


def test_algorithmic_bytes_of_the_316_workload():
    # 52 B per node (x, v read and written, inverse mass) + 20 B per spring
    n = 316
    springs = 6 * n * n - 10 * n + 2
    assert springs == 595978
    assert bench.algorithmic_bytes_per_substep(n * n, springs) == 52 * 99856 + 20 * 595978


def test_collision_bytes_count_each_touched_array_once():
    # 36 B per distinct candidate triangle, 4 B per reference of a queried non-empty cell,
    # 8 B per queried non-empty cell; node-level totals do not enter
    vol = {"cells": 10, "cell_refs": 300, "candidate_tris": 40, "node_queries": 999,
           "refs_tested": 12345, "box_hits": 777}
    assert bench.collision_bytes(vol) == 36 * 40 + 4 * 300 + 8 * 10


def test_median_window_and_roofline():
    w = [(0.5, 1.0), (0.1, 2.0), (0.3, 3.0), (0.2, 4.0), (0.4, 5.0)]
    assert bench.median_window(w) == (0.3, 3.0)
    r = bench.roofline("k", 8e6, 1e-6)
    assert r["achieved"] == pytest.approx(8000.0) and r["frac"] == pytest.approx(1.0)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["traffic"] is None


def test_adjoint_bytes_exceed_two_forward_passes():
    n, s, coll = 4096, 23938, 1e5
    fwd = bench.algorithmic_bytes_per_substep(n, s) + coll
    assert bench.adjoint_bytes_per_substep(n, s, coll) > 2 * fwd


def test_parse_launch():
    from paper_2507_11794_amd import cloth
    cfg = bench.parse_launch("kernel=tile,tile=128,K=2,block=256,graph=0,hits=16,xcd=4")
    assert cfg == {"kernel": cloth.CLOTH_KERNEL_TILE, "tile_nodes": 128,
                   "substeps_per_launch": 2, "block_threads": 256, "use_graph": 0,
                   "hit_slots": 16, "xcd_runs": 4}
    assert bench.parse_launch("") == {}


def test_counter_traffic_is_reported_only_for_matching_sources_and_launch(monkeypatch, tmp_path):
    rec = {"kernel": "k_grid", "workload": "cloth316_sphere100k", "sources_sha256": "a" * 64,
           "launch": {"kernel": 6, "hit_slots": 32}, "traffic_bytes_per_launch": 123.0}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "counter_traffic.json").write_text(json.dumps([rec]))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "sources_sha256", lambda: "a" * 64)
    launch = {"kernel": 6, "hit_slots": 32, "block_threads": 64}
    assert bench.counter_traffic(launch, "cloth316_sphere100k") == 123.0
    assert bench.counter_traffic(launch, "batch512") is None
    assert bench.counter_traffic(dict(launch, hit_slots=16), "cloth316_sphere100k") is None
    assert bench.counter_traffic(dict(launch, kernel=1), "cloth316_sphere100k") is None
    monkeypatch.setattr(bench, "sources_sha256", lambda: "0" * 64)
    assert bench.counter_traffic(launch, "cloth316_sphere100k") is None


def test_sources_hash_follows_the_kernel_sources(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2507_11794_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "a.hip").write_text("kernel A\n")
    (csrc / "b.h").write_text("header\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.sources_sha256()
    (csrc / "a.hip").write_text("kernel A changed\n")
    h1 = bench.sources_sha256()
    (csrc / "README.txt").write_text("not a source\n")
    assert h0 != h1 and bench.sources_sha256() == h1


if __name__ == "__main__":
    sys.exit(pytest.main([__file__, "-q"]))
