"""GPU parity: the HIP library (through its C ABI) against the CPU oracle,
bit for bit (all of the arithmetic is integer)."""
import contextlib

import numpy as np
import pytest

import oracle
from paper_2010_10055_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return "cuda:0"


@pytest.fixture(scope="module")
def lib():
    _dev()
    import paper_2010_10055_amd as pkg
    return pkg


@contextlib.contextmanager
def tuned(pkg, **kw):
    old = pkg.get_tuning()
    pkg.set_tuning(**kw)
    try:
        yield
    finally:
        pkg.set_tuning(**old)


def _np(t):
    return t.cpu().numpy()


def assert_overlap_equal(C, ref, tag=""):
    torch.cuda.synchronize()
    assert np.array_equal(_np(C.rowptr), ref.rowptr), f"{tag} rowptr"
    assert np.array_equal(_np(C.col), ref.col), f"{tag} col"
    assert np.array_equal(_np(C.count), ref.count), f"{tag} count"
    assert np.array_equal(_np(C.seed), ref.seed), f"{tag} seed"


def assert_csr_equal(S, ref, tag=""):
    torch.cuda.synchronize()
    assert np.array_equal(_np(S.rowptr), ref.rowptr), f"{tag} rowptr"
    assert np.array_equal(_np(S.col), ref.col), f"{tag} col"
    assert np.array_equal(_np(S.val), ref.val), f"{tag} val"


def _run_overlap(pkg, A, ms):
    print(f"overlap n={A.nrows} m={A.ncols} nnz={A.nnz} min_shared={ms}", flush=True)
    C = pkg.overlap(pkg.CSRTensors.from_numpy(A, _dev()), ms)
    return C


# ---------------------------------------------------------------------------
# Overlap
# ---------------------------------------------------------------------------

# bits_max_words: 8192 = bitmap path for these sets, 0 = hash path only
PATHS = [pytest.param(8192, id="bitmap"), pytest.param(0, id="hash")]


@pytest.mark.parametrize("bits", PATHS)
def test_overlap_tiny_workload(lib, bits):
    w = synth.make_workload("tiny")
    with tuned(lib, bits_max_words=bits):
        C = _run_overlap(lib, w.A, w.min_shared)
        st = lib.last_stats()
    assert_overlap_equal(C, oracle.overlap(w.A, w.min_shared), "tiny")
    assert st["products"] == synth.overlap_products(w.A)


@pytest.mark.parametrize("bits", PATHS)
@pytest.mark.parametrize("seed,n,m,density,ms", [
    (1, 300, 2000, 0.01, 1), (2, 500, 800, 0.02, 2), (3, 64, 64, 0.3, 1), (4, 1, 5, 0.6, 1),
    (5, 257, 4097, 0.004, 3), (6, 1000, 30000, 0.001, 1), (7, 200, 300, 0.05, 4), (8, 150, 200, 0.08, 6),
])
def test_overlap_random(lib, seed, n, m, density, ms, bits):
    rng = np.random.default_rng(seed)
    A = synth.random_a(rng, n, m, density)
    with tuned(lib, bits_max_words=bits):
        C = _run_overlap(lib, A, ms)
    assert_overlap_equal(C, oracle.overlap(A, ms), f"random{seed}")


@pytest.mark.parametrize("m", [pytest.param(3840 * (1 << 13), id="two-level-widest"),
                               pytest.param(3840 * (1 << 13) + 1, id="three-level-narrowest"),
                               pytest.param((1 << 27) + 17, id="three-level-129-segments"),
                               pytest.param(3840 * (1 << 17) + 5, id="three-level-480-segments")])
def test_overlap_very_wide_transpose(lib, m):
    """Very wide A: up to 3840 buckets of 2^13 columns the transpose takes two
    levels; one column more and it partitions into segments of 2^20 columns
    first, then every segment into buckets of 2^12 columns (three levels)."""
    rng = np.random.default_rng(21)
    n = 400
    rows, cols = [], []
    shared = rng.choice(m, 300, replace=False)   # k-mers that several reads share
    for i in range(n):
        c = np.unique(np.concatenate([rng.choice(shared, 6), rng.integers(0, m, 4), [m - 1] if i % 50 == 0 else []]))
        rows.append(np.full(c.size, i)); cols.append(c)
    rows, cols = np.concatenate(rows), np.concatenate(cols).astype(np.int32)
    vals = rng.integers(0, 10000, rows.size).astype(np.int32)
    A = synth.coo_to_csr(n, m, rows, cols, vals)
    assert_overlap_equal(_run_overlap(lib, A, 1), oracle.overlap(A, 1), f"wide transpose m={m}")


def test_overlap_many_short_rows(lib):
    """Many short rows (0-2 entries) over 2^24 columns."""
    rng = np.random.default_rng(22)
    n, m = 90000, 1 << 24
    per = rng.integers(0, 3, n)
    rows = np.repeat(np.arange(n), per)
    cols = rng.integers(0, 1 << 14, rows.size) * 1024 + rng.integers(0, 2, rows.size)
    key = np.unique(rows.astype(np.int64) * m + cols)   # one entry per (read, k-mer)
    rows, cols = key // m, key % m
    A = synth.coo_to_csr(n, m, rows, cols.astype(np.int32), rng.integers(0, 5000, rows.size).astype(np.int32))
    assert_overlap_equal(_run_overlap(lib, A, 1), oracle.overlap(A, 1), "wide partition")


def test_overlap_wide_partition_several_chunks_per_workgroup(lib):
    """About 1.2e8 columns and 9e6 entries: the transpose partition takes two
    chunks per workgroup so that its (bucket, workgroup) count table stays
    small beside A."""
    rng = np.random.default_rng(23)
    n, per, m = 20000, 470, 3800 << 15
    pool = rng.choice(m, 6000, replace=False)          # k-mers shared by several reads
    rows = np.repeat(np.arange(n, dtype=np.int64), per)
    cols = rng.integers(0, m, rows.size)
    shared = rng.random(rows.size) < 0.02
    cols[shared] = rng.choice(pool, int(shared.sum()))
    key = np.unique(rows * m + cols)
    rows, cols = key // m, key % m
    A = synth.coo_to_csr(n, m, rows, cols.astype(np.int32), rng.integers(0, 30000, rows.size).astype(np.int32))
    assert_overlap_equal(_run_overlap(lib, A, 1), oracle.overlap(A, 1), "multi-chunk partition")


def _sliced_a(rng, n, m):
    """Rows of four kinds over m columns: spread over all of them, confined
    to one narrow range (one slice), empty, and one entry at column m - 1;
    a pool of shared columns gives every kind overlaps."""
    pool = np.unique(np.concatenate([rng.choice(m, 400, replace=False), [0, m - 1]]))
    rows, cols = [], []
    for i in range(n):
        kind = i % 7
        if kind == 0:
            c = np.zeros(0, np.int64)
        elif kind == 1:
            lo = int(rng.integers(0, m - 3000))
            c = lo + rng.choice(3000, 25, replace=False)
        elif kind == 2:
            c = np.array([m - 1])
        else:
            c = np.concatenate([rng.choice(pool, 12), rng.integers(0, m, int(rng.integers(1, 90)))])
        c = np.unique(c)
        rows.append(np.full(c.size, i)); cols.append(c)
    rows, cols = np.concatenate(rows), np.concatenate(cols).astype(np.int32)
    return synth.coo_to_csr(n, m, rows, cols, rng.integers(0, 20000, rows.size).astype(np.int32))


@pytest.mark.parametrize("m", [pytest.param((1 << 23) - 1, id="unsliced-narrow"), pytest.param(1 << 23, id="8-slices"),
                               pytest.param(5 * (1 << 23) + 3, id="24-slices"), pytest.param(1 << 27, id="64-slices"),
                               pytest.param((1 << 27) + 1, id="72-slices"), pytest.param((1 << 27) + (1 << 26) + 5,
                                                                                      id="104-slices")])
def test_overlap_sliced_segments(lib, m):
    """From 2^23 columns the segment pass runs per column slice (rounds of 8
    slices of at most 2^21 columns); one column fewer and it runs per row."""
    A = _sliced_a(np.random.default_rng(31), 3001, m)
    assert_overlap_equal(_run_overlap(lib, A, 1), oracle.overlap(A, 1), f"sliced m={m}")
    assert_overlap_equal(_run_overlap(lib, A, 2), oracle.overlap(A, 2), f"sliced m={m} ms 2")


def test_overlap_unsliced_when_slice_tables_outgrow_a(lib):
    """3e5 rows of one entry over 2^27 columns: the slice tables (2 * 64 + 1
    int32 per row) would outgrow max(4 nnz, 2^24) entries, so the segment
    pass runs per row."""
    rng = np.random.default_rng(33)
    n, m = 300000, 1 << 27
    cols = rng.integers(0, 1 << 12, n) * (m >> 12) + rng.integers(0, 3, n)   # few distinct columns: overlaps
    A = synth.coo_to_csr(n, m, np.arange(n), cols.astype(np.int32), rng.integers(0, 9000, n).astype(np.int32))
    assert_overlap_equal(_run_overlap(lib, A, 1), oracle.overlap(A, 1), "unsliced many rows")


def test_overlap_batched_sliced_segments(lib):
    """Sets of 6e6, 2e3 and 6e6 columns: together they are wide enough for
    the sliced segment pass, whose slices then cut across sets."""
    rng = np.random.default_rng(32)
    sets = [_sliced_a(rng, 700, 6000000), synth.random_a(rng, 60, 2000, 0.01), _sliced_a(rng, 900, 6000001)]
    Cs = lib.overlap_batched([lib.CSRTensors.from_numpy(a, _dev()) for a in sets], [1, 1, 2])
    for s, (a, ms) in enumerate(zip(sets, [1, 1, 2])):
        assert_overlap_equal(Cs[s], oracle.overlap(a, ms), f"set {s}")


def test_overlap_empty_rows_and_matrix(lib):
    A = synth.CSR(4, 7, np.zeros(5, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32))
    C = _run_overlap(lib, A, 1)
    assert C.nnz == 0 and np.all(_np(C.rowptr) == 0)
    rng = np.random.default_rng(8)
    A2 = synth.random_a(rng, 50, 100, 0.05)
    keep = np.ones(50, bool)
    keep[::3] = False   # blank every third row
    rows = np.repeat(np.arange(50), np.diff(A2.rowptr))
    sel = keep[rows]
    A3 = synth.coo_to_csr(50, 100, rows[sel], A2.col[sel], A2.val[sel])
    assert_overlap_equal(_run_overlap(lib, A3, 1), oracle.overlap(A3, 1), "blank rows")


@pytest.mark.parametrize("n,m", [(0, 0), (0, 5), (1, 1), (3, 0)])
def test_overlap_degenerate_shapes(lib, n, m):
    if n and m:
        A = synth.CSR(n, m, np.array([0, 1], np.int64), np.zeros(1, np.int32), np.array([7], np.int32))
    else:
        A = synth.CSR(n, m, np.zeros(n + 1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32))
    C = _run_overlap(lib, A, 1)
    assert_overlap_equal(C, oracle.overlap(A, 1), f"{n}x{m}")


@pytest.mark.parametrize("bits", PATHS)
def test_overlap_adversarial_dense(lib, bits):
    rng = np.random.default_rng(9)
    # one k-mer in every read, one read with every k-mer
    A = synth.random_a(rng, 700, 900, 0.01, dense_rows=[17], dense_cols=[3, 500])
    for ms in (1, 2):
        with tuned(lib, bits_max_words=bits):
            C = _run_overlap(lib, A, ms)
        assert_overlap_equal(C, oracle.overlap(A, ms), f"dense ms={ms}")


def test_overlap_esc_and_overflow_paths(lib):
    rng = np.random.default_rng(10)
    A = synth.random_a(rng, 3000, 400, 0.02, dense_cols=[7, 8])
    ref = oracle.overlap(A, 1)
    # numeric LDS tables for at most 256 distinct columns: larger rows go to
    # ESC; symbolic tables of 256 then 1024 slots: rows with > 768 distinct
    # overflow both and need the third sync
    with tuned(lib, sym_first_log2=8, sym_max_log2=10, num_max_entries=256, bits_max_words=0):
        C = _run_overlap(lib, A, 1)
        st = lib.last_stats()
    assert st["esc_rows"] > 0
    assert st["host_syncs"] == 3
    assert_overlap_equal(C, ref, "esc")
    # bitmap path: no overflow, rows with more than 256 output entries go to ESC
    with tuned(lib, num_max_entries=256):
        C = _run_overlap(lib, A, 1)
        st = lib.last_stats()
    assert st["esc_rows"] > 0
    assert st["host_syncs"] == 2
    assert_overlap_equal(C, ref, "esc bitmap")


def test_overlap_esc_rows_with_two_pair_columns(lib):
    """Rows whose output exceeds the numeric tables go through
    expand-sort-compress while many of their columns hold exactly two pairs
    (carried inline, not gathered): the expansion must give both products of
    such an entry, each with its position."""
    rng = np.random.default_rng(33)
    n, pool = 600, 50
    rows, cols = [], []
    for i in range(n):
        own = [pool + 3 * i + q for q in range(3)]                            # shared with the next read only
        prev = [pool + 3 * ((i - 1) % n) + q for q in range(3)]
        c = np.unique(np.concatenate([own, prev, rng.choice(pool, 40, replace=False)]))
        rows.append(np.full(c.size, i)); cols.append(c)
    m = pool + 3 * n
    rows, cols = np.concatenate(rows), np.concatenate(cols).astype(np.int32)
    A = synth.coo_to_csr(n, m, rows, cols, rng.integers(0, 50000, rows.size).astype(np.int32))
    ref = oracle.overlap(A, 1)
    with tuned(lib, num_max_entries=256):
        C = _run_overlap(lib, A, 1)
        st = lib.last_stats()
    assert st["esc_rows"] > 0
    assert_overlap_equal(C, ref, "esc with two-pair columns")
    assert_overlap_equal(_run_overlap(lib, A, 2), oracle.overlap(A, 2), "two-pair columns, min_shared 2")


@pytest.mark.parametrize("bits", PATHS)
@pytest.mark.parametrize("block", [64, 128, 512])
def test_overlap_launch_shapes_give_same_bits(lib, block, bits):
    w = synth.make_workload("tiny")
    ref = oracle.overlap(w.A, 1)
    with tuned(lib, sym_block=block, num_block=block, sym_first_log2=8, load_pct=50, bits_max_words=bits):
        assert_overlap_equal(_run_overlap(lib, w.A, 1), ref, f"block {block}")


def test_overlap_batched_equals_solo(lib):
    sets = [synth.make_workload("tiny", seed=1000 + s).A for s in range(3)]
    rng = np.random.default_rng(11)
    sets.append(synth.CSR(0, 0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32)))
    sets.append(synth.random_a(rng, 40, 30, 0.2))
    ms = [1, 2, 1, 1, 3]
    # bits_max_words=2: the 40-read set takes the bitmap path, the 200-read
    # sets the hash path, in the same launches
    for bits in (8192, 2, 0):
        with tuned(lib, bits_max_words=bits):
            Cs = lib.overlap_batched([lib.CSRTensors.from_numpy(a, _dev()) for a in sets], ms)
        for s, (a, m) in enumerate(zip(sets, ms)):
            assert_overlap_equal(Cs[s], oracle.overlap(a, m), f"set {s} bits {bits}")


def test_overlap_deterministic(lib):
    w = synth.make_workload("tiny", seed=77)
    A = lib.CSRTensors.from_numpy(w.A, _dev())
    C1 = lib.overlap(A, 1)
    C2 = lib.overlap(A, 1)
    torch.cuda.synchronize()
    for f in ("rowptr", "col", "count", "seed"):
        assert torch.equal(getattr(C1, f), getattr(C2, f))


def test_calls_from_two_threads_on_two_streams(lib):
    """Two host threads, each on its own stream, run overlap and reduction
    calls on different inputs at the same time; every result matches the
    oracle."""
    import threading
    ws = [synth.make_workload("tiny", seed=900 + t) for t in range(2)]
    refs = [(oracle.overlap(w.A, 1), oracle.transitive_reduce(w.R, w.fuzz)) for w in ws]
    errors = []

    def work(t):
        try:
            dev = _dev()
            stream = torch.cuda.Stream(device=dev)
            A = lib.CSRTensors.from_numpy(ws[t].A, dev)
            R = lib.CSRTensors.from_numpy(ws[t].R, dev)
            stream.wait_stream(torch.cuda.current_stream(dev))   # the uploads
            with torch.cuda.stream(stream):
                for rep in range(6):
                    C = lib.overlap(A, 1)
                    S, it = lib.transitive_reduce(R, ws[t].fuzz)
                    stream.synchronize()
                    (cref, (sref, it_ref, _)) = refs[t]
                    assert np.array_equal(_np(C.col), cref.col) and np.array_equal(_np(C.seed), cref.seed)
                    assert np.array_equal(_np(S.col), sref.col) and np.array_equal(_np(S.val), sref.val)
                    assert it == it_ref
        except Exception as e:   # reported by the main thread
            errors.append(f"thread {t}: {e!r}")

    threads = [threading.Thread(target=work, args=(t,)) for t in range(2)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=120)
    assert not any(th.is_alive() for th in threads), "a thread did not finish"
    assert not errors, errors


@pytest.mark.parametrize("case", ["unsorted", "colrange", "negative", "rowptr", "overlap_rows", "min_shared"])
def test_overlap_rejects_malformed(lib, case):
    rng = np.random.default_rng(12)
    A = synth.random_a(rng, 20, 50, 0.2)
    rowptr, col, val, ms = A.rowptr.copy(), A.col.copy(), A.val.copy(), 1
    if case == "unsorted":
        r = int(np.argmax(np.diff(rowptr)))
        a = rowptr[r]
        col[a], col[a + 1] = col[a + 1], col[a]
    elif case == "colrange":
        col[3] = 50
    elif case == "negative":
        val[5] = -1
    elif case == "rowptr":
        rowptr[-2] = rowptr[-1] + 5     # row ranges past nnz and decreasing
    elif case == "overlap_rows":
        rowptr[5] = rowptr[9]           # row 4 covers rows 5..8 too: more entries than A holds
    else:
        ms = 0
    bad = synth.CSR(20, 50, rowptr, col, val)
    with pytest.raises(lib.DibellaError) as ei:
        _run_overlap(lib, bad, ms)
    assert ei.value.status == -1


def test_overlap_batched_rejects_one_malformed_set(lib):
    rng = np.random.default_rng(21)
    sets = [synth.random_a(rng, 20 + 5 * s, 50, 0.2) for s in range(4)]
    bad = sets[2]
    col = bad.col.copy()
    col[3] = 50                                   # column out of range in set 2 only
    sets_bad = sets[:2] + [synth.CSR(bad.nrows, 50, bad.rowptr, col, bad.val)] + sets[3:]
    print("overlap batch of 4, set 2 malformed", flush=True)
    with pytest.raises(lib.DibellaError) as ei:
        lib.overlap_batched([lib.CSRTensors.from_numpy(a, _dev()) for a in sets_bad], [1] * 4)
    assert ei.value.status == -1 and "set 2" in str(ei.value)
    # the library keeps no state from the rejected call
    Cs = lib.overlap_batched([lib.CSRTensors.from_numpy(a, _dev()) for a in sets], [1] * 4)
    for s, a in enumerate(sets):
        assert_overlap_equal(Cs[s], oracle.overlap(a, 1), f"set {s}")


# ---------------------------------------------------------------------------
# Transitive reduction
# ---------------------------------------------------------------------------

def _run_tr(pkg, R, fuzz, **kw):
    print(f"tr n={R.nrows} nnz={R.nnz} fuzz={fuzz} {kw}", flush=True)
    return pkg.transitive_reduce(pkg.CSRTensors.from_numpy(R, _dev()), fuzz, **kw)


@pytest.mark.parametrize("policy", ["edges", "reads"])
@pytest.mark.parametrize("variant,rule", [("A", "row"), ("B", "row"), ("A", "edge"), ("B", "edge")])
def test_tr_tiny_workload(lib, policy, variant, rule):
    w = synth.make_workload("tiny", policy=policy)
    S, it = _run_tr(lib, w.R, w.fuzz, variant=variant, rule=rule)
    ref, it_ref, trace = oracle.transitive_reduce(w.R, w.fuzz, variant, rule)
    assert_csr_equal(S, ref, f"{policy} {variant} {rule}")
    assert it == it_ref
    st = lib.last_stats()
    assert st["nnz_trace"] == list(trace)
    assert st["host_syncs"] == max(1, (it + 1) // 2)  # one per two passes (validity read with the first)


@pytest.mark.parametrize("graph", [False, True])
def test_tr_noisy_tiny(lib, graph):
    w = synth.make_workload("tiny")
    rng = np.random.default_rng(13)
    Rn = synth.perturb_graph(rng, w.R, jitter=60, false_edges=500, flip_codes=0.05)
    for variant in ("A", "B"):
        S, it = _run_tr(lib, Rn, w.fuzz, variant=variant, graph=graph)
        ref, it_ref, _ = oracle.transitive_reduce(Rn, w.fuzz, variant)
        assert_csr_equal(S, ref, f"noisy {variant}")
        assert it == it_ref


@pytest.mark.parametrize("seed", range(6))
def test_tr_random(lib, seed):
    rng = np.random.default_rng(200 + seed)
    n = int(rng.integers(5, 300))
    R = synth.random_r(rng, n, float(rng.uniform(0.01, 0.2)), max_overhang=200,
                       allow_nonpositive=True)
    fuzz = int(rng.integers(0, 100))
    S, it = _run_tr(lib, R, fuzz)
    ref, it_ref, _ = oracle.transitive_reduce(R, fuzz)
    assert_csr_equal(S, ref, f"random {seed}")
    assert it == it_ref


def test_tr_long_rows_global_path(lib):
    rng = np.random.default_rng(14)
    n = 1500
    R = synth.random_r(rng, n, 0.01, max_overhang=300)
    # two hub rows longer than the LDS cap
    rows, cols, vals = [], [], []
    for hub in (5, 900):
        cs = np.setdiff1d(rng.choice(n, 800, replace=False), [hub])
        rows += [hub] * cs.size
        cols += cs.tolist()
        vals += synth.encode_r(rng.integers(1, 300, cs.size), rng.integers(0, 2, cs.size),
                               rng.integers(0, 2, cs.size)).tolist()
    base_rows = np.repeat(np.arange(n), np.diff(R.rowptr))
    keep = ~np.isin(base_rows, [5, 900])
    Rb = synth.coo_to_csr(n, n, np.concatenate([base_rows[keep], rows]),
                          np.concatenate([R.col[keep], cols]), np.concatenate([R.val[keep], vals]))
    ref, it_ref, _ = oracle.transitive_reduce(Rb, 50)
    with tuned(lib, tr_lds_cap=512):
        S, it = _run_tr(lib, Rb, 50)
    assert_csr_equal(S, ref, "hubs")
    assert it == it_ref


@pytest.mark.parametrize("case", ["0x0", "empty", "all-contained", "single-edge"])
def test_tr_degenerate_inputs(lib, case):
    if case == "0x0":
        R = synth.CSR(0, 0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32))
    elif case == "empty":
        R = synth.CSR(5, 5, np.zeros(6, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32))
    elif case == "all-contained":    # overhang 0 everywhere: everything is dropped first
        R = synth.coo_to_csr(3, 3, [0, 1, 2], [1, 2, 0], [0 << 2, 0 << 2, 0 << 2])
    else:
        R = synth.coo_to_csr(2, 2, [0], [1], [(500 << 2) | 1])
    S, it = _run_tr(lib, R, 1000)
    ref, it_ref, _ = oracle.transitive_reduce(R, 1000)
    assert_csr_equal(S, ref, case)
    assert it == it_ref, (it, it_ref)


@pytest.mark.parametrize("block", [64, 128, 512])
def test_tr_launch_shapes_give_same_bits(lib, block):
    w = synth.make_workload("tiny")
    ref, _, _ = oracle.transitive_reduce(w.R, w.fuzz)
    with tuned(lib, tr_block=block, tr_graph_passes=2):
        S, _ = _run_tr(lib, w.R, w.fuzz, graph=True)
    assert_csr_equal(S, ref, f"block {block}")


def test_tr_one_pass(lib):
    w = synth.make_workload("tiny")
    rng = np.random.default_rng(15)
    Rn = synth.perturb_graph(rng, w.R, jitter=30, false_edges=200)
    S, it = _run_tr(lib, Rn, w.fuzz, max_passes=1)
    assert it == 1
    # expected: R without contained entries, minus the marks of one pass
    oh = Rn.val >> 2
    rows = np.repeat(np.arange(Rn.nrows), np.diff(Rn.rowptr))
    pos = oh > 0
    R0 = synth.coo_to_csr(Rn.nrows, Rn.nrows, rows[pos], Rn.col[pos], Rn.val[pos])
    mark = oracle.tr_pass_marks(R0, w.fuzz)
    rows0 = np.repeat(np.arange(R0.nrows), np.diff(R0.rowptr))
    k = mark == 0
    exp = synth.coo_to_csr(R0.nrows, R0.nrows, rows0[k], R0.col[k], R0.val[k])
    assert_csr_equal(S, exp, "one pass")


def test_tr_batched_equals_solo(lib):
    Rs = [synth.make_workload("tiny", seed=1000 + s).R for s in range(3)]
    rng = np.random.default_rng(16)
    Rs.append(synth.random_r(rng, 60, 0.1, allow_nonpositive=True))
    Rs.append(synth.CSR(0, 0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32)))
    fz = [1000, 500, 0, 20, 7]
    for graph in (False, True):
        Ss, its = lib.transitive_reduce_batched([lib.CSRTensors.from_numpy(r, _dev()) for r in Rs], fz,
                                                graph=graph)
        for s, (r, f) in enumerate(zip(Rs, fz)):
            ref, it_ref, _ = oracle.transitive_reduce(r, f)
            assert_csr_equal(Ss[s], ref, f"set {s}")
            assert its[s] == it_ref


@pytest.mark.parametrize("case", ["diagonal", "unsorted", "colrange", "bigoverhang", "fuzz"])
def test_tr_rejects_malformed(lib, case):
    rng = np.random.default_rng(17)
    R = synth.random_r(rng, 30, 0.2)
    col, val, fuzz = R.col.copy(), R.val.copy(), 10
    r = int(np.argmax(np.diff(R.rowptr)))
    a = int(R.rowptr[r])
    if case == "diagonal":
        col[a] = r
        col[a:R.rowptr[r + 1]] = np.sort(col[a:R.rowptr[r + 1]])
    elif case == "unsorted":
        col[a], col[a + 1] = col[a + 1], col[a]
    elif case == "colrange":
        col[a] = 30
    elif case == "bigoverhang":
        val[a] = (1 << 28) << 2          # overhang 2^28 does not fit the packed key
    else:
        fuzz = -1
    bad = synth.CSR(30, 30, R.rowptr, col, val)
    with pytest.raises(lib.DibellaError) as ei:
        _run_tr(lib, bad, fuzz)
    assert ei.value.status == -1


@pytest.mark.parametrize("graph", [False, True])
def test_tr_batched_rejects_one_malformed_set(lib, graph):
    rng = np.random.default_rng(22)
    Rs = [synth.random_r(rng, 30 + 4 * s, 0.2) for s in range(4)]
    bad = Rs[2]
    r = int(np.argmax(np.diff(bad.rowptr)))
    col = bad.col.copy()
    a, b = int(bad.rowptr[r]), int(bad.rowptr[r + 1])
    col[a] = r                                    # a diagonal entry in set 2 only
    col[a:b] = np.sort(col[a:b])
    Rs_bad = Rs[:2] + [synth.CSR(bad.nrows, bad.ncols, bad.rowptr, col, bad.val)] + Rs[3:]
    print(f"tr batch of 4, set 2 malformed, graph={graph}", flush=True)
    with pytest.raises(lib.DibellaError) as ei:
        lib.transitive_reduce_batched([lib.CSRTensors.from_numpy(x, _dev()) for x in Rs_bad], [10] * 4, graph=graph)
    assert ei.value.status == -1 and "set 2" in str(ei.value)
    Ss, its = lib.transitive_reduce_batched([lib.CSRTensors.from_numpy(x, _dev()) for x in Rs], [10] * 4,
                                            graph=graph)
    for s, x in enumerate(Rs):
        ref, it_ref, _ = oracle.transitive_reduce(x, 10)
        assert_csr_equal(Ss[s], ref, f"set {s}")
        assert its[s] == it_ref


def test_timing_records_only_selected_labels(lib):
    from paper_2010_10055_amd import _lib
    w = synth.make_workload("tiny", seed=31)
    A = lib.CSRTensors.from_numpy(w.A, _dev())
    R = lib.CSRTensors.from_numpy(w.R, _dev())
    ref = oracle.overlap(w.A, w.min_shared)
    Sref, _, _ = oracle.transitive_reduce(w.R, w.fuzz)
    print("timing: all labels, then numeric_phase only", flush=True)
    try:
        _lib.timing_enable(True)
        C = lib.overlap(A, w.min_shared)
        S, _ = lib.transitive_reduce(R, w.fuzz)
        every = _lib.timing_collect()
        for name in ("keys", "segments", "numeric_phase", "tr_mark", "tr_compact"):
            assert every[name][1] > 0, name
        assert_overlap_equal(C, ref, "all labels")
        assert_csr_equal(S, Sref, "all labels")

        _lib.timing_select(["numeric_phase"])
        for _ in range(2):
            C = lib.overlap(A, w.min_shared)
            S, _ = lib.transitive_reduce(R, w.fuzz)
        only = _lib.timing_collect()
        assert only["numeric_phase"][1] == 2 and only["numeric_phase"][0] > 0
        assert all(v[1] == 0 for k, v in only.items() if k != "numeric_phase"), only
        assert_overlap_equal(C, ref, "numeric_phase only")
        assert_csr_equal(S, Sref, "numeric_phase only")
    finally:
        _lib.timing_enable(False)
        _lib.timing_select(None)
