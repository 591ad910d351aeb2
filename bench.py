"""Throughput of the two semiring sparse products on one MI355X.

A step is one pass of the whole hot path over one read set:
    C = A A^T            (overlap: count + two seeds, LDS-hash / ESC SpGEMM)
    S = TR(R)            (transitive reduction to the fixed point)
on the mid-size long-read workload (10 Mbp genome with 300 copies of a 2 kbp
repeat at 1% divergence, 30x lognormal reads of mean 10 kbp, 15% error,
k = 17, reliable k-mers in [2, 30], min_shared 2, fuzz 1000).  Inputs are
resident in HBM before timing starts.

value = semiring products per second = (A A^T multiplies + walks examined by
all reduction passes) / step time.  The JSON line also carries the roofline
of the dominant kernel (measured with HIP events on the library's stream,
over the timed steps) and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash(*names) -> str:
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2010_10055_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def phase_bytes(w, C_nnz, products, tr_stats):
    """Algorithmic bytes per step of each timed phase (CSR Gustavson model)."""
    n, nnzA = w.A.nrows, w.A.nnz
    numeric = 8 * n + 8 * nnzA + 16 * nnzA + 8 * products + 24 * C_nnz
    symbolic = 8 * n + 20 * nnzA + 4 * products + 8 * n
    transpose = 8 * nnzA * 2 + 8 * nnzA + 4 * w.A.ncols * 2
    trace = tr_stats["nnz_trace"]
    trip = tr_stats["triples_trace"]
    mark = sum(16 * trace[p] + 8 * trip[p] for p in range(len(trip)))
    compact = sum(8 * trace[p] + 8 * trace[p + 1] for p in range(len(trip)))
    return {"numeric": numeric, "symbolic": symbolic, "transpose": transpose,
            "tr_mark": mark, "tr_compact": compact}


def load_traffic(kernel: str, workload: str, src_hash: str):
    """HBM bytes per step from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source."""
    path = os.path.join(PROFILES, f"{kernel}_{workload}_pmc.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("source_hash") != src_hash:
        return None
    return d.get("hbm_bytes_per_step")


def cpu_baseline(w, budget_s: float):
    """Oracle (plain C, one thread) on a bounded sample of the same workload:
    the overlap rows of a prefix of reads, then the full reduction of R if it
    fits the remaining budget."""
    import numpy as np
    import oracle
    from paper_2010_10055_amd import synth
    A = w.A
    a = np.bincount(A.col, minlength=A.ncols).astype(np.int64)
    row_products = np.add.reduceat(a[A.col], A.rowptr[:-1]) if A.nnz else np.zeros(A.nrows, np.int64)
    row_products[np.diff(A.rowptr) == 0] = 0
    # calibrate on a few rows, then size the sample to ~budget/2 seconds
    t0 = time.perf_counter()
    oracle.overlap(A, w.min_shared, rows=np.arange(min(50, A.nrows)))
    t_cal = time.perf_counter() - t0
    prod_cal = int(row_products[:min(50, A.nrows)].sum())
    rate = prod_cal / max(t_cal, 1e-6)
    want = rate * budget_s * 0.5
    csum = np.cumsum(row_products)
    nrows = int(min(A.nrows, max(50, np.searchsorted(csum, want) + 1)))
    rows = np.arange(nrows)
    t0 = time.perf_counter()
    oracle.overlap(A, w.min_shared, rows=rows)
    t_ov = time.perf_counter() - t0
    prod = int(row_products[:nrows].sum())
    t0 = time.perf_counter()
    _, _, _, walks = oracle.transitive_reduce(w.R, w.fuzz, with_walks=True)
    t_tr = time.perf_counter() - t0
    value = (prod + walks) / (t_ov + t_tr)
    return {"value": value, "unit": "products/s", "cores": 1, "kind": "oracle",
            "sample": f"A*A^T rows 0..{nrows - 1} of {A.nrows} ({prod} products, {t_ov:.1f} s) + "
                      f"full reduction of R ({w.R.nnz} entries, {walks} walks, {t_tr:.1f} s); "
                      f"plain C -O2, single thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="mid", choices=["tiny", "mid", "large"])
    ap.add_argument("--graph", action="store_true", help="run reduction passes as captured HIP graphs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--check", action="store_true", help="compare one step with the oracle first")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2010_10055_amd as db
    from paper_2010_10055_amd import _lib, synth

    dev = "cuda:0"
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    log(f"generating workload '{args.workload}' ...")
    w = synth.make_workload(args.workload, device=dev)
    log(f"  {time.perf_counter() - t0:.1f} s: reads {w.A.nrows}, k-mers {w.A.ncols}, "
        f"nnz(A) {w.A.nnz}, nnz(R) {w.R.nnz}")
    products = synth.overlap_products(w.A)
    A = db.CSRTensors.from_numpy(w.A, dev)
    R = db.CSRTensors.from_numpy(w.R, dev)
    torch.cuda.synchronize()

    def step():
        C = db.overlap(A, w.min_shared)
        S, it = db.transitive_reduce(R, w.fuzz, graph=args.graph)
        return C, S, it

    if args.check:
        import oracle
        C, S, it = step()
        ref = oracle.overlap(w.A, w.min_shared)
        ok = (np.array_equal(C.col.cpu().numpy(), ref.col) and
              np.array_equal(C.seed.cpu().numpy(), ref.seed))
        Sref, it_ref, _ = oracle.transitive_reduce(w.R, w.fuzz)
        ok = ok and np.array_equal(S.col.cpu().numpy(), Sref.col) and it == it_ref
        log(f"check vs oracle: {'ok' if ok else 'MISMATCH'}")
        if not ok:
            sys.exit(1)

    log(f"warmup {args.warmup} ...")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    _lib.timing_enable(True)
    log(f"timing {args.steps} steps ...")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        C, S, it = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    phases = _lib.timing_collect()
    _lib.timing_enable(False)
    tr_stats = db.last_stats()          # last call = the reduction
    db.overlap(A, w.min_shared)
    ov_stats = db.last_stats()
    torch.cuda.synchronize()
    triples = tr_stats["triples"]
    ms_step = elapsed * 1e3 / args.steps
    per_step_products = products + triples
    value = per_step_products / (elapsed / args.steps)

    # roofline of the dominant kernel (largest measured time per step)
    pb = phase_bytes(w, C.nnz, products, tr_stats)
    per_step_ms = {k: v[0] / args.steps for k, v in phases.items() if v[1] > 0}
    dominant = max((k for k in per_step_ms if k in pb), key=lambda k: per_step_ms[k])
    dom_ms = per_step_ms[dominant]
    achieved = pb[dominant] / (dom_ms * 1e-3) / 1e9
    src = {"numeric": ("overlap.hip",), "symbolic": ("overlap.hip",), "transpose": ("overlap.hip",),
           "tr_mark": ("tr.hip",), "tr_compact": ("tr.hip", "runtime.hip")}[dominant]
    traffic = load_traffic(dominant, args.workload, source_hash(*src))
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": dominant, "algorithmic_bytes_per_step": pb[dominant],
                "ms_per_step": round(dom_ms, 4),
                "records_per_step": phases[dominant][1] / args.steps}

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(w, args.cpu_budget)

    out = {
        "metric": "semiring products/s (A*A^T multiplies + transitive-reduction walks)",
        "value": value, "unit": "products/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": args.workload, "reads": w.A.nrows, "kmers": w.A.ncols,
                   "nnz_A": w.A.nnz, "overlap_products": products, "nnz_C": C.nnz,
                   "min_shared": w.min_shared, "nnz_R": w.R.nnz, "nnz_S": S.nnz,
                   "tr_passes": it, "tr_walks": triples, "fuzz": w.fuzz, "graph": args.graph,
                   "parallelism": "single GPU"},
        "phases_ms_per_step": {k: round(v, 4) for k, v in per_step_ms.items()},
        "overlap_products_per_s": products / (sum(per_step_ms.get(k, 0) for k in
                                                  ("transpose", "symbolic", "numeric", "esc")) * 1e-3),
        "host_syncs": {"overlap": ov_stats["host_syncs"], "tr": tr_stats["host_syncs"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
