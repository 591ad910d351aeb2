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


def test_results_compared_element_by_element_not_by_sums():
    """A result whose columns are permuted within a row (equal sums, equal
    sizes) or whose values moved between entries is rejected; an identical
    one is accepted."""
    import torch
    from paper_2010_10055_amd._lib import CSRTensors, OverlapCSR
    rowptr = torch.tensor([0, 3, 5])
    col = torch.tensor([1, 4, 7, 0, 2], dtype=torch.int32)
    cnt = torch.tensor([3, 1, 2, 5, 5], dtype=torch.int32)
    seed = torch.arange(20, dtype=torch.int32).view(5, 4)
    C = OverlapCSR(2, 2, rowptr, col, cnt, seed)
    S = CSRTensors(2, 2, rowptr, col, cnt)
    ref = autotune.snapshot(([C], [S], [2]))
    same = OverlapCSR(2, 2, rowptr.clone(), col.clone(), cnt.clone(), seed.clone())
    assert autotune.results_equal(ref, ([same], [S], [2]))
    perm = OverlapCSR(2, 2, rowptr, torch.tensor([4, 1, 7, 0, 2], dtype=torch.int32), cnt, seed)
    assert int(perm.col.sum()) == int(col.sum())
    assert not autotune.results_equal(ref, ([perm], [S], [2]))
    moved = OverlapCSR(2, 2, rowptr, col, torch.tensor([1, 3, 2, 5, 5], dtype=torch.int32), seed)
    assert not autotune.results_equal(ref, ([moved], [S], [2]))
    assert not autotune.results_equal(ref, ([C], [S], [3]))            # pass count differs
    assert not autotune.results_equal(ref, ([C], [S]))                 # missing output
    assert not autotune.results_equal(ref, ([C], [S], [2.0 + 1]))
    # the snapshot is a copy: overwriting the live tensors later does not change it
    col[0] = 9
    assert int(ref[3][0]) == 1                 # leaves: nrows, ncols, rowptr, col, ...
    assert not autotune.results_equal(ref, ([C], [S], [2]))
