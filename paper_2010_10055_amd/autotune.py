"""Autotuner for the library's launch shapes and table sizes.

A workload class is the GPU architecture plus coarse statistics of the
inputs (read count, k-mer entries per read, min_shared, number of sets).
For a class the tuner runs a coordinate search over the tunable fields of
dibella_tuning: every candidate configuration is timed on the caller's
workload (median of a few runs on the device) and must reproduce the
results of the starting configuration bit for bit (every output tensor
equal element by element, every other output value equal), otherwise it is
rejected.  The best configuration per class is kept in a JSON cache
(path: $DIBELLA_TUNING_CACHE, else ~/.cache/dibella/tuning.json).
"""
from __future__ import annotations

import json
import math
import os
import statistics
import time
from typing import Callable, Dict, Iterable, List, Optional, Sequence

SEARCH_SPACE: Dict[str, List[int]] = {
    "bits_max_words": [8192, 0],
    "sym_block": [128, 256, 512],
    "num_block": [128, 256, 512],
    "load_pct": [50, 65, 75, 85],
    "sym_first_log2": [10, 11, 12, 13],
    "tr_block": [128, 256, 512],
    "tr_lds_cap": [1024, 4096],
    "tr_graph_passes": [2, 4, 8],
}


def cache_path() -> str:
    p = os.environ.get("DIBELLA_TUNING_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "dibella", "tuning.json")


def _bucket(x: float) -> int:
    return int(math.floor(math.log2(max(1.0, float(x)))))


def workload_key(arch: str, sets: Sequence, min_shared: Sequence[int]) -> str:
    """Class of a workload: arch, log2 buckets of total reads and of A entries
    per read, the min_shared values and the log2 bucket of the set count."""
    reads = sum(int(a.nrows) for a in sets)
    nnz = sum(int(a.nnz) for a in sets)
    per_read = nnz / max(1, reads)
    ms = "-".join(str(m) for m in sorted(set(int(x) for x in min_shared)))
    return f"{arch}|reads2^{_bucket(reads)}|ent2^{_bucket(per_read)}|ms{ms}|sets2^{_bucket(len(sets))}"


def load_cache(path: Optional[str] = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict, path: Optional[str] = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + f".tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def leaves(result) -> list:
    """Every tensor and plain value in a result, in a fixed order: lists,
    tuples, dicts and dataclasses (OverlapCSR, CSRTensors) are walked
    recursively."""
    import dataclasses
    out = []

    def walk(x):
        if isinstance(x, (list, tuple)):
            for y in x:
                walk(y)
        elif isinstance(x, dict):
            for k in sorted(x):
                walk(x[k])
        elif dataclasses.is_dataclass(x) and not isinstance(x, type):
            for f in dataclasses.fields(x):
                walk(getattr(x, f.name))
        else:
            out.append(x)
    walk(result)
    return out


def snapshot(result) -> list:
    """A copy of a result's leaves that later calls cannot overwrite."""
    return [x.clone() if hasattr(x, "clone") else x for x in leaves(result)]


def results_equal(ref: list, result) -> bool:
    """True if `result` has the same leaves as the snapshot `ref`: tensors of
    equal dtype, shape and elements, other values equal."""
    import torch
    got = leaves(result)
    if len(got) != len(ref):
        return False
    for a, b in zip(ref, got):
        if isinstance(a, torch.Tensor) or isinstance(b, torch.Tensor):
            if not (isinstance(a, torch.Tensor) and isinstance(b, torch.Tensor)):
                return False
            if a.dtype != b.dtype or a.shape != b.shape or not torch.equal(a, b):
                return False
        elif a != b:
            return False
    return True


def coordinate_search(start: dict, space: Dict[str, Iterable[int]], measure: Callable[[dict], Optional[float]],
                      budget_s: float = 60.0, rounds: int = 2, log: Callable[[str], None] = lambda s: None):
    """Greedy coordinate descent.  measure(cfg) returns seconds, or None if
    cfg is invalid or gives different results.  Returns (best cfg, best time,
    number of evaluations)."""
    t_end = time.perf_counter() + budget_s
    best = dict(start)
    best_t = measure(best)
    if best_t is None:
        raise RuntimeError("the starting configuration failed")
    evals = 1
    for _ in range(rounds):
        improved = False
        for field, values in space.items():
            for v in values:
                if time.perf_counter() > t_end:
                    return best, best_t, evals
                if best.get(field) == v:
                    continue
                cand = dict(best)
                cand[field] = v
                t = measure(cand)
                evals += 1
                if t is not None and t < best_t * 0.98:
                    log(f"  {field}={v}: {t * 1e3:.3f} ms (was {best_t * 1e3:.3f})")
                    best, best_t, improved = cand, t, True
        if not improved:
            break
    return best, best_t, evals


def autotune(run: Callable[[], object], key: str, budget_s: float = 60.0, repeats: int = 3,
             space: Optional[Dict[str, Iterable[int]]] = None, cache_file: Optional[str] = None,
             force: bool = False, log: Callable[[str], None] = print) -> dict:
    """Tune the library for `run` (a callable doing the work on the device
    and returning its outputs) and store the result under `key`.  Every
    candidate's outputs must equal the starting configuration's bit for bit
    (results_equal), else the candidate is rejected."""
    import torch
    import paper_2010_10055_amd as db
    cache = load_cache(cache_file)
    if not force and key in cache:
        cfg = cache[key]["tuning"]
        db.set_tuning(**cfg)
        return cfg
    start = db.get_tuning()
    ref = snapshot(run())
    torch.cuda.synchronize()

    def measure(cfg):
        try:
            db.set_tuning(**cfg)
        except Exception:
            return None
        try:
            got = run()
            torch.cuda.synchronize()
            if not results_equal(ref, got):
                log(f"  rejected {cfg}: results differ")
                return None
            ts = []
            for _ in range(repeats):
                t0 = time.perf_counter()
                run()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            return statistics.median(ts)
        except db.DibellaError:
            return None

    best, best_t, evals = coordinate_search(start, space or SEARCH_SPACE, measure, budget_s, log=log)
    db.set_tuning(**best)
    cache[key] = {"tuning": best, "ms": best_t * 1e3, "evaluations": evals,
                  "default_ms": None, "when": time.strftime("%Y-%m-%dT%H:%M:%S")}
    save_cache(cache, cache_file)
    return best


def apply_cached(key: str, cache_file: Optional[str] = None) -> Optional[dict]:
    """Apply the cached configuration of `key` if there is one."""
    import paper_2010_10055_amd as db
    ent = load_cache(cache_file).get(key)
    if not ent:
        return None
    db.set_tuning(**ent["tuning"])
    return ent["tuning"]
