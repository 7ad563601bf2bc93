"""The synthetic workloads against the sizes the paper prints (tests/golden/paper_sizes.json).
The paper rounds to one or two significant digits ("4K", "100K"); a stand-in matches when it
lies within 2.5 % of the printed figure (4,096 nodes print as 4K)."""
import json
import os

from paper_2507_11794_amd import workloads as W

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_sizes.json")))


def _close(ours, key):
    printed = GOLDEN[key]["value"]
    return abs(ours - printed) <= 0.025 * printed


def test_hanging_cloth_at_the_no_collision_limit():
    assert W.config2().n_nodes == GOLDEN["cloth_nodes_no_collision_max"]["value"]


def test_differentiable_scene_cloth_is_the_4k_resolution():
    inp, _ = W.config4()
    assert _close(inp.n_nodes, "cloth_nodes_dragon_30fps")


def test_benchmark_cloth_and_surface_match_the_100k_scene():
    V, T = W.geodesic_sphere(71)  # the benchmark surface's mesh (before displacement)
    assert _close(316 * 316, "cloth_nodes_100k_collision")
    assert _close(T.shape[0], "dragon_triangles") and _close(V.shape[0], "dragon_vertices")
