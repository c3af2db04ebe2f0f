"""Host logic of the autotuner (no GPU): coordinate descent finds the minimum of a
separable cost and of a cost with one interaction, evaluates each setting once, and the
JSON cache round-trips; the workload key and the stencil-size estimate behave."""
import numpy as np

from paper_2401_08586_amd import autotune as A
from paper_2401_08586_amd import workloads as W


def test_descent_separable_minimum():
    space = {"a": [1, 2, 3, 4, 5], "b": [10, 20, 30], "c": [0, 1]}
    calls = []

    def cost(p):
        calls.append(p)
        return (p["a"] - 4) ** 2 + (p["b"] - 20) ** 2 / 100 + (0.5 if p["c"] else 0.0)

    best, val, n = A.coordinate_descent(cost, space=space, start={"a": 1, "b": 10, "c": 1})
    assert best == {"a": 4, "b": 20, "c": 0} and val == 0.0
    keys = [tuple(sorted(p.items())) for p in calls]
    assert len(keys) == len(set(keys)) == n  # every setting timed once


def test_descent_interaction_needs_second_sweep():
    space = {"x": [0, 1, 2], "y": [0, 1, 2]}
    table = {(0, 0): 5, (1, 0): 4, (2, 0): 6, (1, 1): 3, (1, 2): 7, (0, 1): 9, (2, 1): 1, (0, 2): 9, (2, 2): 9}
    best, val, _ = A.coordinate_descent(lambda p: table[(p["x"], p["y"])], space=space, start={"x": 0, "y": 0})
    assert (best["x"], best["y"]) == (2, 1) and val == 1


def test_cache_roundtrip(tmp_path):
    path = str(tmp_path / "tune.json")
    c = A.Cache(path)
    assert c.get("k") is None
    c.put("k", {"block_target": 48}, 1.5)
    c2 = A.Cache(path)
    assert c2.get("k") == {"block_target": 48}
    assert c2.data["k"]["ms"] == 1.5


def test_workload_key_and_stencil_sizes():
    lat = W.lattice(3, 20, 0.05, 0.1, seed=1)
    mean, p99 = A.stencil_sizes([lat], sample=2000)
    # 2.4^3 = 13.8 particles per cell; interior stencils hold 27 cells' worth
    assert 250 < mean < 400 and p99 <= 27 * 30
    cl = W.clustered(20000, 3, dim=3)
    mean2, p99b = A.stencil_sizes([cl], sample=2000)
    assert p99b / mean2 > p99 / mean  # clustering spreads the stencil sizes
    k1 = A.workload_key("gfx950", 3, 0, [lat.n], p99, mean)
    k2 = A.workload_key("gfx950", 3, 0, [cl.n], p99b, mean2)
    assert k1 != k2 and k1.startswith("gfx950|d3|m0|")
    assert A.workload_key("gfx950", 3, 0, [1100, 1000], 1, 1) == A.workload_key("gfx950", 3, 0, [1200, 1000], 1, 1)
    assert np.isfinite(mean)
