"""Throughput of the two semiring sparse products on one MI355X.

A step is one pass of the whole hot path over one read set:
    C = A A^T            (overlap: count + two seeds, LDS-hash / ESC SpGEMM)
    S = TR(R)            (transitive reduction to the fixed point)
on one GPU's share of a large run by default (50 Mbp genome with 5% repeats
from 1-6 kbp families at 0.5-3% divergence, 40x lognormal reads of mean
12 kbp, 12% error, k = 17, reliable k-mers in [2, 40], min_shared 2; R = the
true overlaps of at least 1 kbp among the candidate pairs of C, fuzz 1000).
Inputs are resident in HBM before timing starts.

value = semiring products per second = (A A^T multiplies + walks examined by
all reduction passes) / step time.  The JSON line also carries the roofline
of the dominant kernel (measured with HIP events on the library's stream,
over the timed steps), the CPU oracle timed on bounded samples, the
batching comparison (64 uneven sets, graph-captured reductions) and the
serving comparison (continuous batching vs FIFO on the same trace).
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


def kernel_bytes(w, C_nnz, products, tr_stats):
    """Algorithmic bytes per step of each timed kernel.  The two products use
    the CSR Gustavson model of a row-wise SpGEMM (symbolic: row pointers, A
    columns and the column's A^T segment per entry, 4 B per product;
    numeric: the same plus A values, 8 B per product and 24 B per output
    entry); every partition pass of the transpose moves what a pass over
    12-byte (column, read|position) pairs must (12 B in, 12 B out; its count
    pass reads the 4-byte keys) and the last pass also writes 8 B per column
    record; a reduction pass reads a row-pointer pair per entry and 8 B per
    walk."""
    n, nnzA, m = w.A.nrows, w.A.nnz, w.A.ncols
    trace = tr_stats["nnz_trace"]
    trip = tr_stats["triples_trace"]
    sym = 8 * n + 20 * nnzA + 4 * products + 8 * n
    return {
        "keys": 8 * n + 8 * nnzA + 12 * nnzA,
        "part_count": 4 * nnzA,
        "part_scatter": 24 * nnzA,
        "part2_count": 4 * nnzA,
        "part2_scatter": 24 * nnzA,
        "bucket_sort": 24 * nnzA + 8 * m,
        "segments": 16 * n + 20 * nnzA,
        "sym_bits": sym,
        "sym_hash": sym,
        "numeric": 8 * n + 8 * nnzA + 16 * nnzA + 8 * products + 24 * C_nnz,
        "tr_mark": sum(16 * trace[p] + 8 * trip[p] for p in range(len(trip))),
        "tr_compact": sum(9 * trace[p] + 8 * trace[p + 1] for p in range(len(trip))),
    }


KERNEL_SOURCES = {"keys": ("overlap.hip",), "part_count": ("overlap.hip",), "part_scatter": ("overlap.hip",),
                  "bucket_sort": ("overlap.hip",), "part2_count": ("overlap.hip",), "part2_scatter": ("overlap.hip",),
                  "segments": ("overlap.hip",), "sym_bits": ("overlap.hip",),
                  "sym_hash": ("overlap.hip",), "numeric": ("overlap.hip",), "esc": ("overlap.hip",),
                  "tr_mark": ("tr.hip",), "tr_compact": ("tr.hip",)}


def load_traffic(kernel: str, workload: str, src_hash: str, profiles: str = PROFILES):
    """HBM bytes per launch (per phase for the numeric phase) from the
    committed rocprofv3 counter summary, if it was taken on the current
    kernel source."""
    phase = kernel == "numeric_phase"
    path = os.path.join(profiles, f"{'numeric' if phase else kernel}_{workload}_pmc.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("source_hash") != src_hash:
        return None
    return d.get("hbm_bytes_per_phase" if phase else "hbm_bytes_per_launch")


# the kernels of each timed unit (a unit of several kernels sums them per call)
KERNEL_NAMES = {"keys": ("k_ov_keys",), "part_count": ("k_ov_part_count<false>",),
                "part_scatter": ("k_ov_part_scatter<false",), "part2_count": ("k_ov_part_count<true>",),
                "part2_scatter": ("k_ov_part_scatter<true",), "bucket_sort": ("k_ov_bucket_sort",),
                "segments": ("k_ov_seg_slices", "k_ov_scatter"),
                "sym_bits": ("k_ov_sym_bits",), "sym_hash": ("k_ov_sym_hash",), "numeric": ("k_ov_numeric",),
                "tr_mark": ("k_tr_mark",), "tr_compact": ("k_tr_compact",)}
CALIB_BYTES = 1 << 30


# reference kernels of libdibella_calib.so: (name, bytes read, bytes written)
# per launch as the access pattern fixes them; a 4-byte touch per 64- or
# 128-byte line and a random 4-byte gather count as 4 bytes each
CALIB_GATHERS = 1 << 24
CALIB_CASES = (("k_calib_read", CALIB_BYTES, 0), ("k_calib_write", 0, CALIB_BYTES),
               ("k_calib_copy", CALIB_BYTES, CALIB_BYTES),
               ("k_calib_stride<64>", CALIB_BYTES // 64 * 4, 0), ("k_calib_stride<128>", CALIB_BYTES // 128 * 4, 0),
               ("k_calib_gather", CALIB_GATHERS * 4, 0))


def calib_copy():
    """Plain device kernels of known traffic, the references for scaling HBM
    counters (libdibella_calib.so, built beside the library): a 1 GiB read,
    a 1 GiB write, a 1 GiB copy, one 4-byte read per 64 bytes and per 128
    bytes over 1 GiB, and 2^24 random 4-byte gathers over 4 GiB.  Prints the
    time of each (best of three)."""
    import ctypes
    import torch
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2010_10055_amd", "libdibella_calib.so"))
    V, I64, I32, U64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64
    lib.calib_read.argtypes = [V, I64, V, V]
    lib.calib_write.argtypes = [V, I64, V]
    lib.calib_copy.argtypes = [V, V, I64, V]
    lib.calib_stride.argtypes = [V, I64, I32, V, V]
    lib.calib_gather.argtypes = [V, I64, I64, U64, V, V]
    dev = "cuda:0"
    x = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    big = torch.ones(4 * CALIB_BYTES // 4, dtype=torch.float32, device=dev)
    out = torch.zeros(1, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream().cuda_stream
    cases = [("read", lambda: lib.calib_read(x.data_ptr(), CALIB_BYTES, out.data_ptr(), st)),
             ("write", lambda: lib.calib_write(y.data_ptr(), CALIB_BYTES, st)),
             ("copy", lambda: lib.calib_copy(x.data_ptr(), y.data_ptr(), CALIB_BYTES, st)),
             ("stride64", lambda: lib.calib_stride(x.data_ptr(), CALIB_BYTES, 64, out.data_ptr(), st)),
             ("stride128", lambda: lib.calib_stride(x.data_ptr(), CALIB_BYTES, 128, out.data_ptr(), st)),
             ("gather4GiB", lambda: lib.calib_gather(big.data_ptr(), 4 * CALIB_BYTES, CALIB_GATHERS, 12345,
                                                     out.data_ptr(), st))]
    res = {}
    for name, fn in cases:
        best = None
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            if fn() != 0:
                raise RuntimeError(f"calibration kernel {name} failed")
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        res[name] = round(best, 4)
        log(f"  calib {name}: {best:.3f} ms")
    print(json.dumps({"calib_bytes": CALIB_BYTES, "calib_gathers": CALIB_GATHERS, "ms": res}), flush=True)


def _csv_rows(d, suffix):
    import csv
    import glob
    out = []
    for f in glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True):
        with open(f) as fh:
            out.extend(csv.DictReader(fh))
    return out


def _counter_per_kernel(d, counter):
    """{kernel name: [value per dispatch]} for one counter (KiB for the TCC
    size counters) from a rocprofv3 --pmc CSV directory."""
    per = {}
    for r in _csv_rows(d, "counter_collection.csv"):
        if r.get("Counter_Name") != counter:
            continue
        per.setdefault(r.get("Kernel_Name", ""), []).append(float(r["Counter_Value"]))
    return per


def summarize_profiles(trace_dir, fetch_dir, write_dir, cfetch_dir, cwrite_dir, workload, command,
                       out_dir: str = PROFILES):
    """Write the profiles/ summaries: per-kernel durations of the timed run
    (rocprofv3 kernel stats) and, per main kernel, HBM bytes per launch from
    FETCH_SIZE / WRITE_SIZE scaled by the counters of the calibration copy."""
    import statistics
    os.makedirs(out_dir, exist_ok=True)
    stats = _csv_rows(trace_dir, "kernel_stats.csv")
    lines = [f"# rocprofv3 kernel statistics, workload '{workload}'", f"# command: {command}",
             f"{'kernel':64s} {'calls':>6s} {'total_ms':>10s} {'avg_us':>10s} {'pct':>6s}"]
    rows = sorted(stats, key=lambda r: -float(r.get("TotalDurationNs", 0)))
    ours = [r for r in rows if "dibella::" in r.get("Name", "")]
    others = [r for r in rows if "dibella::" not in r.get("Name", "")]

    def row_line(r):
        name = r.get("Name", "")[:64]
        return (f"{name:64s} {int(r['Calls']):6d} {float(r['TotalDurationNs']) / 1e6:10.3f} "
                f"{float(r['AverageNs']) / 1e3:10.2f} {float(r.get('Percentage', 0)):6.2f}")
    lines.append("## library kernels (all)")
    lines.extend(row_line(r) for r in ours)
    lines.append("## other kernels (workload generation, torch plumbing; largest 10)")
    lines.extend(row_line(r) for r in others[:10])
    # per call of the library: k_ov_write_rowptr runs once per overlap call,
    # k_tr_init_state once per reduction call
    def calls_of(marker):
        return sum(int(r["Calls"]) for r in ours if marker in r["Name"])
    n_ov, n_tr = calls_of("k_ov_write_rowptr"), calls_of("k_tr_init_state")
    if n_ov or n_tr:
        lines.append("")
        lines.append(f"## timed units, kernel time per call ({n_ov} overlap calls, {n_tr} reduction calls)")
        lines.append(f"{'unit':14s} {'kernels':44s} {'launches/call':>13s} {'ms/call':>9s}")
        for label, knames in KERNEL_NAMES.items():
            n = n_tr if label.startswith("tr_") else n_ov
            hit = [r for r in ours if any(k in r["Name"] for k in knames)]
            if not hit or not n:
                continue
            tot = sum(float(r["TotalDurationNs"]) for r in hit)
            launches = sum(int(r["Calls"]) for r in hit)
            note = "  (launches overlap: the phase span is below)" if label == "numeric" else ""
            lines.append(f"{label:14s} {'+'.join(knames):44s} {launches / n:13.1f} {tot / n / 1e6:9.3f}{note}")
    # the numeric phase of one call: its k_ov_numeric launches overlap on
    # several streams; its span runs from the first start to the last end
    # among the launches that follow one k_ov_write_rowptr
    spans, group, nlaunch = [], None, []
    for r in sorted(_csv_rows(trace_dir, "kernel_trace.csv"), key=lambda r: int(r["Start_Timestamp"])):
        name = r["Kernel_Name"]
        if "k_ov_write_rowptr" in name:
            if group:
                spans.append(group[1] - group[0])
                nlaunch.append(group[2])
            group = [None, None, 0]
        elif "k_ov_numeric" in name and group is not None:
            t0, t1 = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
            group = [t0 if group[0] is None else min(group[0], t0), t1 if group[1] is None else max(group[1], t1),
                     group[2] + 1]
    if group and group[0] is not None:
        spans.append(group[1] - group[0])
        nlaunch.append(group[2])
    if spans:
        lines.append("")
        lines.append(f"numeric phase (k_ov_numeric launches of one call, overlapping on 3 streams): "
                     f"{len(spans)} calls, {statistics.mean(nlaunch):.1f} launches per call, "
                     f"span avg_us {statistics.mean(spans) / 1e3:.2f}")
    with open(os.path.join(out_dir, f"kernels_{workload}_trace.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    cf = _counter_per_kernel(cfetch_dir, "FETCH_SIZE")
    cw = _counter_per_kernel(cwrite_dir, "WRITE_SIZE")

    def ref(per, name):
        """Mean counter bytes per dispatch of one calibration kernel."""
        v = [x for n, vals in per.items() if name + "(" in n or n.endswith(name) for x in vals]
        return statistics.mean(v) * 1024 if v else 0.0
    # reads and writes are scaled by what the counters read for the plain
    # copy kernel (1 GiB read, 1 GiB written); the other reference kernels
    # are recorded beside it
    copy_fetch, copy_write = ref(cf, "k_calib_copy"), ref(cw, "k_calib_copy")
    f_fetch = copy_fetch / CALIB_BYTES if copy_fetch else None
    f_write = copy_write / CALIB_BYTES if copy_write else None
    refs = {}
    for name, rd, wr in CALIB_CASES:
        fb_, wb_ = ref(cf, name), ref(cw, name)
        refs[name] = {"read_bytes": rd, "write_bytes": wr, "FETCH_SIZE_bytes": fb_, "WRITE_SIZE_bytes": wb_,
                      "fetch_factor": round(fb_ / rd, 4) if rd else None,
                      "write_factor": round(wb_ / wr, 4) if wr else None}
    print("calibration: " + ", ".join(f"{k} FETCH {v['fetch_factor']} WRITE {v['write_factor']}"
                                      for k, v in refs.items()))
    fetch = _counter_per_kernel(fetch_dir, "FETCH_SIZE")
    write = _counter_per_kernel(write_dir, "WRITE_SIZE")
    calls = sum(len(v) for n, v in fetch.items() if "k_ov_write_rowptr" in n)   # overlap calls profiled
    for label, knames in KERNEL_NAMES.items():
        per_f = [[x for n, v in fetch.items() if k in n for x in v] for k in knames]
        per_w = [[x for n, v in write.items() if k in n for x in v] for k in knames]
        present = [i for i in range(len(knames)) if per_f[i] and per_w[i]]
        if not present or not f_fetch or not f_write:
            continue
        fv = [x for i in present for x in per_f[i]]
        wv = [x for i in present for x in per_w[i]]
        # one dispatch of each kernel of the unit per call
        fb = sum(statistics.mean(per_f[i]) for i in present) * 1024 / f_fetch
        wb = sum(statistics.mean(per_w[i]) for i in present) * 1024 / f_write
        kname = "+".join(knames[i] for i in present)
        d = {"kernel": kname, "workload": workload, "command": command,
             "source_hash": source_hash(*KERNEL_SOURCES[label]),
             "fetch_KiB_per_call_raw": fb * f_fetch / 1024, "write_KiB_per_call_raw": wb * f_write / 1024,
             "dispatches": len(per_f[present[0]]), "read_calibration_factor": f_fetch,
             "write_calibration_factor": f_write, "calibration_kernel": "k_calib_copy",
             "reference_kernels": refs, "hbm_bytes_per_launch": fb + wb, "hbm_read_bytes_per_launch": fb, "hbm_write_bytes_per_launch": wb}
        if label == "numeric" and calls:
            # all launches of the phase of one call
            d["overlap_calls"] = calls
            d["hbm_bytes_per_phase"] = (sum(fv) * 1024 / f_fetch + sum(wv) * 1024 / f_write) / calls
        with open(os.path.join(out_dir, f"{label}_{workload}_pmc.json"), "w") as f:
            json.dump(d, f, indent=1)
    print(f"summaries written to {out_dir}")


def summarize_raw(dirs, workload, command, out_dir: str = PROFILES):
    """Write profiles/counters_raw_<workload>.txt: per kernel of the library
    and per calibration kernel, the mean per dispatch of every counter found
    in the given rocprofv3 --pmc CSV directories (raw TCC request counts, to
    check how FETCH_SIZE / WRITE_SIZE weigh requests of each size)."""
    import statistics
    per = {}
    for d in dirs:
        for r in _csv_rows(d, "counter_collection.csv"):
            name = r.get("Kernel_Name", "")
            short = None
            if "k_calib_" in name:
                short = name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")
            if short is None and "dibella::" in name:
                short = name.split("(")[0].replace("void ", "").replace("dibella::", "")
            if short is None:
                continue
            per.setdefault(short, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    names = sorted({c for v in per.values() for c in v})
    known = {n: (rd, wr) for n, rd, wr in CALIB_CASES}
    lines = [f"# rocprofv3 raw counters, mean per dispatch, workload '{workload}'", f"# command: {command}",
             "# reference kernels (bytes read / written as their access pattern fixes them): " +
             ", ".join(f"{n} {rd} / {wr}" for n, (rd, wr) in known.items()),
             f"{'kernel':44s} {'dispatches':>10s} " + " ".join(f"{c:>26s}" for c in names)]
    for k in sorted(per):
        v = per[k]
        nd = max(len(x) for x in v.values())
        lines.append(f"{k[:44]:44s} {nd:10d} " + " ".join(
            f"{statistics.mean(v[c]):26.1f}" if c in v else f"{'-':>26s}" for c in names))
    os.makedirs(out_dir, exist_ok=True)
    path = os.path.join(out_dir, f"counters_raw_{workload}.txt")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"written {path}")


def copy_rate() -> float:
    """GB/s of a 1 GiB device-to-device copy (1 GiB read + 1 GiB written),
    best of five."""
    import torch
    x = torch.ones(CALIB_BYTES // 4, dtype=torch.int32, device="cuda:0")
    y = torch.empty_like(x)
    y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = None
    for _ in range(5):
        e0.record()
        y.copy_(x)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del x, y
    return 2 * CALIB_BYTES / (best * 1e-3) / 1e9


def gather_probe():
    """Random 8-byte gathers (torch indexing: indices read in order, one
    random element each) over arrays from 2 MB to 4 GB: the rate at which the
    GPU serves random lines by footprint.  A footprint within one XCD's L2
    is served several times faster than anything larger; the 256 MB Infinity
    Cache gives random lines no gain over HBM."""
    import torch
    m = 1 << 26
    out = []
    for mb in (2, 8, 32, 128, 256, 512, 1024, 4096):
        n = mb * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.int64, device="cuda:0")
        idx = torch.randint(0, n, (m,), device="cuda:0")
        for _ in range(2):
            a[idx]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        best = None
        for _ in range(5):
            e0.record()
            a[idx]
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        out.append({"array_MB": mb, "ms": round(best, 4), "G_gathers_per_s": round(m / best / 1e6, 2)})
        log(f"  {mb:5d} MB: {m / best / 1e6:7.2f} G random 8-byte gathers/s")
        del a, idx
    print(json.dumps({"gather_probe": out}))


def _row_products(A):
    import numpy as np
    a = np.bincount(A.col, minlength=A.ncols).astype(np.int64)
    rp = np.add.reduceat(a[A.col], A.rowptr[:-1]) if A.nnz else np.zeros(A.nrows, np.int64)
    rp[np.diff(A.rowptr) == 0] = 0
    return rp


def _row_walks(R):
    """Walks i -> k -> j a reduction pass examines per row of R."""
    import numpy as np
    deg = np.diff(R.rowptr).astype(np.int64)
    per_entry = deg[R.col] if R.col.size else np.zeros(0, np.int64)
    out = np.zeros(R.nrows, np.int64)
    if R.col.size:
        nz = deg > 0
        out[nz] = np.add.reduceat(per_entry, R.rowptr[:-1][nz])
    return out


def _spread_rows(weights, want, nblocks=64):
    """About `want` of the total weight in `nblocks` row blocks spread evenly
    over the rows (rows are in random genome order, blocks avoid any bias of
    a prefix)."""
    import numpy as np
    n = weights.size
    total = max(int(weights.sum()), 1)
    frac = min(1.0, want / total)
    rows = []
    for b in range(nblocks):
        lo, hi = b * n // nblocks, (b + 1) * n // nblocks
        cs = np.cumsum(weights[lo:hi])
        take = int(np.searchsorted(cs, cs[-1] * frac if cs.size else 0)) + 1 if cs.size else 0
        rows.append(np.arange(lo, min(hi, lo + max(take, 1))))
    return np.unique(np.concatenate(rows)).astype(np.int64)


def cpu_legs(w, R, tr_stats, budget_s: float, threads: int = 0):
    """The oracle (plain C -O2) on the host's cores, on bounded samples of
    the same step: A^T built once (timed; every oracle row call needs it),
    a sample of A A^T rows spread over the matrix, and one reduction pass
    over a sample of R's rows.  Each rate scales its part of the whole step
    (all products, the walks of all passes); the step estimate is the
    transpose plus both scaled parts.  Single thread: `cpu_baseline`; the
    same with the sampled rows in row ranges on all host cores (threads
    sharing A^T): `cpu_parallel`."""
    import numpy as np
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    A = w.A
    if threads <= 0:
        try:
            threads = len(os.sched_getaffinity(0))
        except AttributeError:
            threads = os.cpu_count() or 1
        threads = max(1, min(16, threads))
    rprod = _row_products(A)
    rwalk = _row_walks(R)
    products = int(rprod.sum())
    walks_all = int(tr_stats["triples"])
    t0 = time.perf_counter()
    at = oracle.transpose(A)
    t_at = time.perf_counter() - t0
    # calibrate the row rate on a few rows, then size the samples
    cal = _spread_rows(rprod, 2e6)
    t0 = time.perf_counter()
    oracle.overlap(A, w.min_shared, rows=cal, at=at)
    rate = max(int(rprod[cal].sum()), 1) / max(time.perf_counter() - t0, 1e-4)
    tcal = _spread_rows(rwalk, 2e6)
    t0 = time.perf_counter()
    oracle.tr_pass_marks(R, w.fuzz, rows=tcal)
    trate = max(int(rwalk[tcal].sum()), 1) / max(time.perf_counter() - t0, 1e-4)
    part = budget_s * 0.3

    def run(nthreads):
        rows = _spread_rows(rprod, rate * part * nthreads)
        trows = _spread_rows(rwalk, trate * part * 0.3 * nthreads)
        chunks = [c for c in np.array_split(rows, nthreads) if c.size]
        tchunks = [c for c in np.array_split(trows, nthreads) if c.size]
        t0 = time.perf_counter()
        with ThreadPoolExecutor(len(chunks)) as ex:
            list(ex.map(lambda r: oracle.overlap(A, w.min_shared, rows=r, at=at), chunks))
        t_rows = time.perf_counter() - t0
        t0 = time.perf_counter()
        with ThreadPoolExecutor(len(tchunks)) as ex:
            list(ex.map(lambda r: oracle.tr_pass_marks(R, w.fuzz, rows=r), tchunks))
        t_tr = time.perf_counter() - t0
        p_s, w_s = int(rprod[rows].sum()), int(rwalk[trows].sum())
        step = t_at + t_rows * products / max(p_s, 1) + t_tr * walks_all / max(w_s, 1)
        return {"value": (products + walks_all) / step, "unit": "products/s", "cores": len(chunks),
                "kind": "oracle",
                "sample": (f"A^T built once in {t_at:.1f} s (single thread); A*A^T rows: {rows.size} of {A.nrows} in "
                           f"64 blocks spread over the matrix ({p_s} of {products} products) in {t_rows:.1f} s; "
                           f"one reduction pass over {trows.size} of {R.nrows} rows of R ({w_s} walks) in "
                           f"{t_tr:.1f} s; whole step scaled by products and by the walks of all {len(tr_stats['triples_trace'])} "
                           f"passes ({walks_all}): {step:.1f} s; plain C -O2, {len(chunks)} thread(s)"),
                "step_s_estimated": round(step, 2)}
    single = run(1)
    multi = run(threads) if threads > 1 else None
    del at
    return single, multi


def batch_compare(db, synth, nsets: int, steps: int, tune_budget: float = 0.0):
    """The batching workload: `nsets` independent read sets (genomes
    log-uniform in 50 kbp..5 Mbp, 10-50x, lognormal reads of mean 8 kbp,
    15% error, k = 17, reliable [2, 8], min_shared 1, fuzz 1000): the plain
    path (one overlap + one reduction call per set, one after the other) and
    the batched path (one batched overlap call and one batched reduction
    call for all sets), same stream.  The reductions run as captured HIP
    graphs (the batching workload's recipe); the same comparison without
    graphs is reported beside it.  Results are compared set by set."""
    import torch
    t0 = time.perf_counter()
    ws = synth.batch_workloads(nsets, device="cuda:0")
    log(f"  batch generation {time.perf_counter() - t0:.1f} s: reads {sum(w.A.nrows for w in ws)}")
    As = [db.CSRTensors.from_numpy(w.A, "cuda:0") for w in ws]
    Rs = [db.CSRTensors.from_numpy(w.R, "cuda:0") for w in ws]
    ms = [w.min_shared for w in ws]
    fz = [w.fuzz for w in ws]
    products = sum(synth.overlap_products(w.A) for w in ws)

    def plain(graph):
        out = []
        for a, r, m, f in zip(As, Rs, ms, fz):
            C = db.overlap(a, m)
            S, it = db.transitive_reduce(r, f, graph=graph)
            out.append((C, S, it))
        return out

    def batched(graph):
        Cs = db.overlap_batched(As, ms)
        Ss, its = db.transitive_reduce_batched(Rs, fz, graph=graph)
        return list(zip(Cs, Ss, its))

    tuned = None
    if tune_budget > 0:
        from paper_2010_10055_amd import autotune
        key = autotune.workload_key("gfx950", [w.A for w in ws], ms)
        t0 = time.perf_counter()
        tuned = autotune.autotune(lambda: batched(True), key, budget_s=tune_budget, repeats=2, log=log)
        log(f"  autotune {time.perf_counter() - t0:.1f} s -> {tuned}")
    from paper_2010_10055_amd import autotune
    ref = autotune.snapshot(plain(True))
    same = autotune.results_equal(ref, batched(True)) and autotune.results_equal(ref, batched(False))
    torch.cuda.synchronize()
    times = {}
    for name, fn, graph in (("plain", plain, True), ("batched", batched, True),
                            ("plain_no_graph", plain, False), ("batched_no_graph", batched, False)):
        fn(graph)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn(graph)
        torch.cuda.synchronize()
        times[name] = (time.perf_counter() - t0) / steps
    return {"sets": nsets, "reads": sum(w.A.nrows for w in ws), "overlap_products": products, "graph": True,
            "plain_ms": round(times["plain"] * 1e3, 3), "batched_ms": round(times["batched"] * 1e3, 3),
            "speedup": round(times["plain"] / times["batched"], 3), "bit_identical": bool(same),
            "no_graph": {"plain_ms": round(times["plain_no_graph"] * 1e3, 3),
                         "batched_ms": round(times["batched_no_graph"] * 1e3, 3),
                         "speedup": round(times["plain_no_graph"] / times["batched_no_graph"], 3)},
            "tuning": tuned}


def main_pool_entry(w_main):
    """The timed step's reads as a layout job: A rebuilt with strand bits in
    its values (what R from C's seeds needs), device resident."""
    import dataclasses
    from paper_2010_10055_amd import serve, synth
    A1, _ = synth.kmer_matrix(w_main.reads, w_main.k, w_main.lo, w_main.hi, device="cuda:0", strand_bit=True)
    return serve.pool_entry(dataclasses.replace(w_main, A=A1), "cuda:0")


def kmer_compare(w, reps: int = 2):
    """A from the timed step's reads on the device (dibella_kmer_matrix):
    best wall time of `reps` builds, the library's per-stage event time, the
    windows per second, and the result checked equal to the generator's A
    (torch: canonical codes, torch.unique, a sort by read), whose time is
    reported beside it."""
    import numpy as np
    import torch
    import paper_2010_10055_amd as db
    from paper_2010_10055_amd import _lib, synth
    bases = torch.as_tensor(w.reads.bases, device="cuda:0")
    offsets = torch.as_tensor(w.reads.offsets, device="cuda:0")
    windows = int(np.maximum(np.diff(w.reads.offsets) - w.k + 1, 0).sum())
    A, codes = db.kmer_matrix(bases, offsets, w.k, w.lo, w.hi)
    torch.cuda.synchronize()
    del A, codes
    best = None
    _lib.timing_enable(True)
    for _ in range(reps):
        t0 = time.perf_counter()
        A, codes = db.kmer_matrix(bases, offsets, w.k, w.lo, w.hi)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
        if _ < reps - 1:
            del A, codes
    ph = _lib.timing_collect()
    _lib.timing_enable(False)
    stages = {k: round(v[0] / reps, 3) for k, v in ph.items() if k.startswith("kmer_") and v[1]}
    same = (A.ncols == w.A.ncols and np.array_equal(A.rowptr.cpu().numpy(), w.A.rowptr) and
            np.array_equal(A.col.cpu().numpy(), w.A.col) and np.array_equal(A.val.cpu().numpy(), w.A.val))
    if not same:
        raise RuntimeError("the library's A differs from the generator's")
    del A, codes
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    synth.kmer_matrix(w.reads, w.k, w.lo, w.hi, device="cuda:0")
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    del bases, offsets
    torch.cuda.empty_cache()
    out = {"reads": int(w.reads.n), "bases": int(len(w.reads.bases)), "windows": windows, "k": w.k,
           "bounds": [w.lo, w.hi], "ms": round(best * 1e3, 2), "stage_ms": stages,
           "windows_per_s": round(windows / best), "equal_to_generator": same,
           "generator_ms": round(t_gen * 1e3, 1)}
    log(f"  {best * 1e3:.1f} ms ({windows / best / 1e9:.2f} G windows/s), stages {stages}; "
        f"generator (torch) {t_gen * 1e3:.0f} ms; A equal")
    return out


# Integer operations of one extension-table cell: compare the two bases,
# pick match or mismatch, three additions (diagonal, and the gap from each
# side), two maxima, one test against the X-drop floor.
ALIGN_OPS_PER_CELL = 8
# Plain vector ALU peak (32-bit integer lane operations): 256 CUs, 4 SIMDs of
# 16 lanes each, 2.4 GHz.
ALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9


def align_compare(inp, reads, rows: int, reps: int = 2, scores=(1, -1, -2, 25), min_score: int = 300):
    """R from the alignment (dibella_r_from_alignment) over the first `rows`
    reads' rows of C (the other rows left empty): best kernel time of
    `reps` calls, the cells of the extension tables considered, cells and
    pairs per second, and the cells' integer operations against the vector
    ALU peak."""
    import torch
    import paper_2010_10055_amd as db
    from paper_2010_10055_amd import _lib
    C = db.overlap(inp.A, inp.min_shared)
    n = C.nrows
    rows = min(rows, n)
    rp = C.rowptr.clone()
    rp[rows + 1:] = rp[rows]
    e = int(rp[rows].item())
    sub = db.OverlapCSR(n, n, rp, C.col[:e].clone(), C.count[:e].clone(), C.seed[:e].clone())
    nnz_c = C.nnz
    del C
    pairs = e - rows                                   # off-diagonal entries (every row has its diagonal)
    bases = torch.as_tensor(reads.bases, device="cuda:0")
    offsets = torch.as_tensor(reads.offsets, device="cuda:0")
    mat, mis, gap, X = scores
    R = db.r_from_alignment(sub, bases, offsets, inp.k, mat, mis, gap, X, min_score)
    torch.cuda.synchronize()
    del R
    best = wall = None
    for _ in range(reps):
        _lib.timing_enable(True)
        t0 = time.perf_counter()
        R = db.r_from_alignment(sub, bases, offsets, inp.k, mat, mis, gap, X, min_score)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ph = _lib.timing_collect()
        _lib.timing_enable(False)
        cells = db.last_stats()["cells"]
        k_ms = ph["align"][0]
        best = k_ms if best is None else min(best, k_ms)
        wall = dt if wall is None else min(wall, dt)
        kept = R.nnz
        del R
    ops = cells * ALIGN_OPS_PER_CELL / (best * 1e-3)
    out = {"rows": rows, "reads": n, "pairs": pairs, "pairs_all_rows": nnz_c - n,
           "scores": {"match": mat, "mismatch": mis, "gap": gap, "xdrop": X, "min_score": min_score},
           "cells": int(cells), "kernel_ms": round(best, 2), "call_ms": round(wall * 1e3, 2),
           "cells_per_s": round(cells / (best * 1e-3)), "pairs_per_s": round(pairs / (best * 1e-3)),
           "kept_pairs": kept,
           "roofline": {"bound": "alu", "achieved": round(ops / 1e12, 3), "peak": round(ALU_PEAK_OPS / 1e12, 2),
                        "unit": "Tops/s (int32 lane operations, 8 per cell)",
                        "frac": round(ops / ALU_PEAK_OPS, 4)}}
    log(f"  {rows} rows, {pairs} pairs, {cells / 1e9:.1f} G cells in {best:.1f} ms "
        f"({cells / (best * 1e-3) / 1e9:.0f} G cells/s, {ops / ALU_PEAK_OPS:.3f} of the ALU peak), "
        f"{kept} pairs kept")
    del bases, offsets, sub
    torch.cuda.empty_cache()
    return out


def blocked_compare(inp, nblocks=(4, 16), reps: int = 2):
    """The overlap graph of one layout job built whole (dibella_overlap, then
    R from C's seeds) and blocked (dibella_overlap_graph_blocked: C formed a
    block of reads at a time): best wall time of `reps` builds and the peak
    device memory the build allocates beyond its inputs; every blocked R is
    checked equal to the whole one."""
    import torch
    import paper_2010_10055_amd as db
    A, L = inp.A, inp.read_len
    rest = (inp.k, inp.min_overlap, inp.max_drift, inp.min_density)

    def whole():
        C = db.overlap(A, inp.min_shared)
        return db.r_from_seeds(C, L, *rest), 1

    def blocked(nb):
        rows = -(-A.nrows // nb)
        return lambda: db.overlap_graph_blocked(A, inp.min_shared, L, *rest, block_rows=rows)

    def measure(fn):
        R, nb = fn()
        torch.cuda.synchronize()
        del R
        best = None
        torch.cuda.reset_peak_memory_stats()
        base = torch.cuda.memory_allocated()
        for _ in range(reps):
            t0 = time.perf_counter()
            R, nb = fn()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
            if _ < reps - 1:
                del R
        peak = torch.cuda.max_memory_allocated() - base
        return R, nb, best, peak

    Rw, _, tw, pw = measure(whole)
    out = {"reads": A.nrows, "nnz_R": Rw.nnz,
           "whole": {"ms": round(tw * 1e3, 2), "peak_gib": round(pw / 2**30, 2)}}
    log(f"  whole: {tw * 1e3:.1f} ms, peak {pw / 2**30:.2f} GiB")
    for nb in nblocks:
        Rb, got, tb, pb = measure(blocked(nb))
        same = all(torch.equal(a, b) for a, b in ((Rb.rowptr, Rw.rowptr), (Rb.col, Rw.col), (Rb.val, Rw.val)))
        if not same:
            raise RuntimeError(f"blocked overlap graph ({nb} blocks) differs from the whole one")
        out[f"blocks_{got}"] = {"ms": round(tb * 1e3, 2), "peak_gib": round(pb / 2**30, 2), "equal_to_whole": same}
        log(f"  {got} blocks: {tb * 1e3:.1f} ms, peak {pb / 2**30:.2f} GiB, R equal to the whole build")
        del Rb
    del Rw
    return out


def serve_compare(w_main, njobs: int, slots: int = 3, seed: int = 5000, main_entry=None):
    """Serving: Poisson streams of layout jobs (overlap, R from C's seeds on
    the device, reduction): 90% of the jobs one of two instances of the
    large workload's recipe (50 Mbp genome, 40x, ~167k reads: the timed
    step's reads and one more seed), 10% of the tiny one, all device
    resident, A with strand bits.  FIFO (one slot: one job on the device at
    a time) and continuous batching (`slots` slots, each a host thread with
    its own stream) replay the same trace, at 0.8x the FIFO capacity
    measured on a probe (latency) and at 1.5x (saturation: throughput).
    Admission budget: the free device memory measured before the runs."""
    import numpy as np
    import torch
    from paper_2010_10055_amd import serve
    t0 = time.perf_counter()
    pool = [main_entry if main_entry is not None else main_pool_entry(w_main)]
    log(f"  pool {w_main.name}#0 from the timed step's reads: footprint {pool[0][2] / 2**30:.2f} GiB")
    pool += serve.make_pool([(w_main.name, 1, seed, 1.0), ("tiny", 4, seed + 100, 1.0)], device="cuda:0", log=log)
    log(f"  serve pool {time.perf_counter() - t0:.1f} s")
    torch.cuda.empty_cache()
    budget = serve.hbm_free_bytes()
    clock = serve.WallClock()
    # FIFO capacity on a probe of the same mix
    probe = serve.draw_jobs(np.random.default_rng(seed), pool, 12, rate=1e9)
    fifo = serve.GpuSlots(1, clock)
    try:
        for j in probe[:3]:
            fifo.submit(j, 0)
            fifo.wait(None)
        t0 = time.perf_counter()
        for j in probe:
            fifo.submit(j, 0)
            fifo.wait(None)
        service = (time.perf_counter() - t0) / len(probe)
    finally:
        fifo.close()
    # work budget: one job that fills the GPU plus small ones beside it
    work_cap = int(1.25 * max(p[3] for p in pool))
    out = {"jobs": njobs, "slots": slots, "fifo_service_ms": round(service * 1e3, 2),
           "hbm_budget_gib": round(budget / 2**30, 1), "work_cap_products": work_cap,
           "job_mix": f"90% {w_main.name} recipe (2 instances), 10% tiny (4 instances); R from C's seeds",
           "r_from_seeds": {"min_overlap": pool[0][1].min_overlap, "max_drift": pool[0][1].max_drift,
                            "min_density_per_10kbp": pool[0][1].min_density}}
    for label, factor in (("load_0.8", 0.8), ("load_1.5", 1.5)):
        rate = factor / service
        jobs = serve.draw_jobs(np.random.default_rng(seed + 1), pool, njobs, rate=rate)
        res = {"rate_jobs_per_s": round(rate, 2)}
        for name, nslots in (("fifo", 1), ("continuous", slots)):
            clock = serve.WallClock()
            ex = serve.GpuSlots(nslots, clock)
            st = {}
            count = [0]

            def progress(d, count=count, name=name):
                count[0] += 1
                if count[0] % 30 == 0:
                    log(f"    {label} {name}: {count[0]} jobs done at {clock.now():.1f} s")
            try:
                done = serve.serve(jobs, ex, clock, hbm_budget=budget, slots=nslots, stats=st, on_done=progress,
                                   work_cap=work_cap)
            finally:
                ex.close()
            s = serve.summarize(done, clock.now())
            s.update(peak_running=st["peak_running"], peak_reserved_gib=round(st["peak_reserved"] / 2**30, 1))
            res[name] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in s.items()}
            log(f"  {label} {name}: {res[name]['jobs_per_s']} jobs/s, p50 {res[name]['p50_ms']} ms, "
                f"p99 {res[name]['p99_ms']} ms")
        res["throughput_ratio"] = round(res["continuous"]["jobs_per_s"] / max(1e-9, res["fifo"]["jobs_per_s"]), 3)
        res["p99_ratio"] = round(res["fifo"]["p99_ms"] / max(1e-9, res["continuous"]["p99_ms"]), 3)
        out[label] = res
    del pool
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large", choices=["tiny", "mid", "large"])
    ap.add_argument("--graph", action="store_true", help="run reduction passes as captured HIP graphs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--check", action="store_true", help="compare one step with the oracle first")
    ap.add_argument("--batch-sets", type=int, default=64, help="sets of the batching comparison (0 = skip)")
    ap.add_argument("--tune-budget", type=float, default=30.0, help="seconds of autotuning for the batch (0 = off)")
    ap.add_argument("--serve-jobs", type=int, default=120, help="jobs of the serving comparison (0 = skip)")
    ap.add_argument("--serve-slots", type=int, default=3, help="slots of continuous batching")
    ap.add_argument("--no-kmer", action="store_true", help="skip the k-mer counting leg")
    ap.add_argument("--align-rows", type=int, default=8192,
                    help="rows of C aligned by the alignment leg (0 = skip)")
    ap.add_argument("--align-scores", type=int, nargs=4, default=[1, -1, -2, 25],
                    metavar=("MATCH", "MISMATCH", "GAP", "XDROP"), help="scores of the alignment leg")
    ap.add_argument("--blocks", type=int, nargs="*", default=[4, 16],
                    help="block counts of the blocked overlap graph comparison (none = skip)")
    ap.add_argument("--calib-copy", action="store_true", help="only run the reference kernels used to scale counters")
    ap.add_argument("--gather-probe", action="store_true", help="only measure random-gather rates by footprint")
    ap.add_argument("--summarize-profiles", nargs=5, metavar=("TRACE", "FETCH", "WRITE", "CFETCH", "CWRITE"),
                    help="write profiles/ summaries from rocprofv3 CSV directories")
    ap.add_argument("--profile-command", default="", help="command recorded in the summaries")
    ap.add_argument("--summarize-raw", nargs="+", metavar="DIR",
                    help="write the raw-counter summary from rocprofv3 --pmc CSV directories")
    args = ap.parse_args()
    if args.summarize_profiles:
        summarize_profiles(*args.summarize_profiles, args.workload, args.profile_command)
        return
    if args.summarize_raw:
        summarize_raw(args.summarize_raw, args.workload, args.profile_command)
        return
    if args.calib_copy:
        calib_copy()
        return
    if args.gather_probe:
        gather_probe()
        return
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
    default_tuning = db.get_tuning()
    t_start = time.perf_counter()
    log(f"generating workload '{args.workload}' ...")
    w = synth.make_workload(args.workload, device=dev)
    products = synth.overlap_products(w.A)
    A = db.CSRTensors.from_numpy(w.A, dev)
    # R: the overlap graph of the true coordinates restricted to the
    # off-diagonal pattern of C (a perfect aligner's verdict on the candidates)
    C0 = db.overlap(A, w.min_shared)
    Rh = synth.restrict_to_pattern(w.R, C0.rowptr, C0.col, device=dev)
    del C0
    R = db.CSRTensors.from_numpy(Rh, dev)
    torch.cuda.synchronize()
    log(f"  {time.perf_counter() - t_start:.1f} s: reads {w.A.nrows}, k-mers {w.A.ncols}, "
        f"nnz(A) {w.A.nnz}, nnz(R) {Rh.nnz} (true overlaps {w.R.nnz}, restricted to the candidates)")

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
        Sref, it_ref, _ = oracle.transitive_reduce(Rh, w.fuzz)
        ok = ok and np.array_equal(S.col.cpu().numpy(), Sref.col) and it == it_ref
        log(f"check vs oracle: {'ok' if ok else 'MISMATCH'}")
        if not ok:
            sys.exit(1)

    def units(phases, nsteps, C, tr_stats):
        """ms and launches per step of every recorded unit, the algorithmic
        bytes of each, and the unit with the largest time."""
        per_step_ms = {k: v[0] / nsteps for k, v in phases.items() if v[1] > 0}
        launches = {k: v[1] / nsteps for k, v in phases.items() if v[1] > 0}
        pb = kernel_bytes(w, C.nnz, products, tr_stats)
        # the numeric launches of one call overlap on several streams: the phase
        # (first launch to last, one record per call) is the unit that is timed
        if "numeric_phase" in per_step_ms and "numeric" in pb:
            pb["numeric_phase"] = pb.pop("numeric")
        dominant = max((k for k in per_step_ms if k in pb), key=lambda k: per_step_ms[k])
        return per_step_ms, launches, pb, dominant

    # every unit's events are recorded over the warmup steps after the first
    # (the per-unit table, and the choice of the dominant unit); the timed
    # steps record only the dominant unit's, so that the events of the other
    # units cost the timed steps no host time
    prof_steps = max(args.warmup - 1, 1) if args.warmup > 0 else 0
    log(f"warmup {args.warmup} ({prof_steps} with every unit timed) ...")
    for i in range(args.warmup):
        if i == args.warmup - prof_steps:
            torch.cuda.synchronize()
            _lib.timing_enable(True)
        C, S, it = step()
    torch.cuda.synchronize()
    if prof_steps:
        unit_phases = _lib.timing_collect()
        _lib.timing_enable(False)
        per_step_ms, launches, pb, dominant = units(unit_phases, prof_steps, C, db.last_stats())
        _lib.timing_select([dominant])
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
    _lib.timing_select(None)
    tr_stats = db.last_stats()          # last call = the reduction
    db.overlap(A, w.min_shared)
    ov_stats = db.last_stats()
    torch.cuda.synchronize()
    triples = tr_stats["triples"]
    ms_step = elapsed * 1e3 / args.steps
    per_step_products = products + triples
    value = per_step_products / (elapsed / args.steps)
    if not prof_steps:
        per_step_ms, launches, pb, dominant = units(phases, args.steps, C, tr_stats)

    # roofline of the dominant kernel, from its events over the timed steps
    if phases[dominant][1] == 0:
        raise RuntimeError(f"no timing records of '{dominant}' over the timed steps")
    dom_ms = phases[dominant][0] / args.steps
    launches = dict(launches, **{dominant: phases[dominant][1] / args.steps})
    achieved = pb[dominant] / (dom_ms * 1e-3) / 1e9
    traffic = load_traffic(dominant, args.workload,
                           source_hash(*KERNEL_SOURCES["numeric" if dominant == "numeric_phase" else dominant]))
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": round(traffic) if traffic else None,
                "traffic_GBps": round(traffic / (dom_ms / launches[dominant] * 1e-3) / 1e9, 1) if traffic else None,
                "kernel": dominant, "launches_per_step": launches[dominant],
                "algorithmic_bytes_per_launch": pb[dominant] / launches[dominant],
                "avg_launch_ms": round(dom_ms / launches[dominant], 4)}
    if dominant == "numeric_phase":
        roofline["kernel_launches_per_phase"] = launches.get("numeric")
    if traffic:
        roofline["overfetch"] = round(traffic / (pb[dominant] / launches[dominant]), 3)
    # what this machine streams (a 1 GiB device copy, read + write) beside the published peak
    roofline["copy_GBps_measured"] = round(copy_rate(), 1)
    kernels = {k: {"ms_per_step": round(per_step_ms[k], 4), "launches_per_step": launches[k],
                   "model_GBps": (round(pb[k] / (per_step_ms[k] * 1e-3) / 1e9, 1) if k in pb else None)}
               for k in per_step_ms}
    kernels_timed_over = (f"{prof_steps} warmup steps (every unit's events)" if prof_steps
                          else f"the {args.steps} timed steps")
    nnz_C = C.nnz
    del C, S
    log(f"  {ms_step:.2f} ms per step, {dominant} {dom_ms:.2f} ms ({achieved / HBM_PEAK_GBS:.3f} of the HBM peak)")

    cpu = cpu_par = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on bounded samples, one thread, then all host cores) ...")
        cpu, cpu_par = cpu_legs(w, Rh, tr_stats, args.cpu_budget)

    batch = None
    if args.batch_sets > 0:
        log(f"batching comparison ({args.batch_sets} sets) ...")
        batch = batch_compare(db, synth, args.batch_sets, max(1, min(args.steps, 5)), args.tune_budget)
        db.set_tuning(**default_tuning)

    kmer = None
    if not args.no_kmer:
        log("A from the reads on the device vs the generator ...")
        kmer = kmer_compare(w)
    served = blocked = align = None
    entry = None
    if args.serve_jobs > 0 or args.blocks or args.align_rows > 0:
        del A, R
        torch.cuda.empty_cache()
        entry = main_pool_entry(w)
    if args.align_rows > 0:
        log(f"R from the alignment ({args.align_rows} rows of C) ...")
        align = align_compare(entry[1], w.reads, args.align_rows, scores=tuple(args.align_scores))
    if args.blocks:
        log(f"blocked overlap graph ({args.blocks} blocks) vs whole ...")
        blocked = blocked_compare(entry[1], tuple(args.blocks))
    if args.serve_jobs > 0:
        log(f"serving comparison ({args.serve_jobs} jobs per run) ...")
        served = serve_compare(w, args.serve_jobs, args.serve_slots, main_entry=entry)

    out = {
        "metric": "semiring products/s (A*A^T multiplies + transitive-reduction walks)",
        "value": value, "unit": "products/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": args.workload, "reads": w.A.nrows, "kmers": w.A.ncols,
                   "nnz_A": w.A.nnz, "overlap_products": products, "nnz_C": nnz_C,
                   "min_shared": w.min_shared, "nnz_R": Rh.nnz, "nnz_S": int(tr_stats["nnz_trace"][-1]),
                   "tr_passes": it, "tr_walks": triples, "fuzz": w.fuzz, "graph": args.graph,
                   "r_recipe": "true overlaps >= 1 kbp restricted to the off-diagonal pattern of C",
                   "parallelism": "single GPU"},
        "kernels": kernels,
        "kernels_timed_over": kernels_timed_over,
        "overlap_products_per_s_gpu_time": products / (sum(
            per_step_ms.get(k, 0) for k in ("keys", "part_count", "part_scatter", "part2_count", "part2_scatter",
                                             "bucket_sort", "segments", "sym_bits", "sym_hash",
                                             "numeric_phase" if "numeric_phase" in per_step_ms else "numeric",
                                             "esc")) * 1e-3),
        "overlap_products_per_s_numeric_phase": (products / (dom_ms * 1e-3) if dominant == "numeric_phase" else
                                                 products / (per_step_ms["numeric_phase"] * 1e-3)
                                                 if "numeric_phase" in per_step_ms else None),
        "tr_walks_per_s_mark": (triples / (per_step_ms["tr_mark"] * 1e-3) if "tr_mark" in per_step_ms else None),
        "tr_nnz_trace": [int(x) for x in tr_stats["nnz_trace"]],
        "host_syncs": {"overlap": ov_stats["host_syncs"], "tr": tr_stats["host_syncs"]},
        "roofline": roofline,
        "batch": batch,
        "kmer_matrix": kmer,
        "blocked": blocked,
        "align": align,
        "serve": served,
        "cpu_baseline": cpu,
        "cpu_parallel": cpu_par,
        "wall_s": round(time.perf_counter() - t_start, 1),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
