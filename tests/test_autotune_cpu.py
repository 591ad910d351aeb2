"""Autotuner logic on the CPU: the coordinate search finds the optimum of a
known cost surface, rejects failing candidates, honours its budget, and the
JSON cache round-trips."""
from paper_2010_10055_amd import autotune


def test_coordinate_search_finds_separable_optimum():
    space = {"a": [1, 2, 3, 4], "b": [10, 20, 30]}

    def cost(cfg):
        return (cfg["a"] - 3) ** 2 + (cfg["b"] - 20) ** 2 / 100.0 + 1.0

    best, t, evals = autotune.coordinate_search({"a": 1, "b": 10}, space, cost, budget_s=10)
    assert best == {"a": 3, "b": 20}
    assert t == 1.0 and evals > 1


def test_rejected_candidates_are_skipped():
    space = {"a": [1, 2, 3]}
    best, _, _ = autotune.coordinate_search({"a": 1}, space, lambda c: None if c["a"] == 3 else 5 - c["a"])
    assert best == {"a": 2}


def test_budget_stops_the_search():
    calls = []

    def cost(cfg):
        calls.append(cfg)
        return 1.0
    autotune.coordinate_search({"a": 0}, {"a": list(range(1000))}, cost, budget_s=0.0)
    assert len(calls) == 1


def test_cache_roundtrip(tmp_path):
    p = str(tmp_path / "t.json")
    autotune.save_cache({"k": {"tuning": {"x": 1}}}, p)
    assert autotune.load_cache(p) == {"k": {"tuning": {"x": 1}}}
    assert autotune.load_cache(str(tmp_path / "missing.json")) == {}


def test_workload_key_buckets():
    from types import SimpleNamespace as N
    k1 = autotune.workload_key("gfx950", [N(nrows=30000, nnz=3.9e7)], [2])
    k2 = autotune.workload_key("gfx950", [N(nrows=31000, nnz=4.0e7)], [2])
    k3 = autotune.workload_key("gfx950", [N(nrows=200, nnz=5e4)], [1])
    assert k1 == k2 != k3
