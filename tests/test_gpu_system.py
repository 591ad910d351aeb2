"""GPU system tests: the mid-size workload against the oracle at full size
(bitmap and hash paths), the large workload at full size against the oracle
(every row of C, the whole reduction), the batching workload (64 sets) in
full, the serving loop (each job's result in the mix equals its solo
result, tolerance 0, and the oracle's), the autotuner (tuned configurations
reproduce the starting configuration's outputs element by element), and
batched graph-captured reductions."""
import numpy as np
import pytest

import oracle
from paper_2010_10055_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def db():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_10055_amd as pkg
    return pkg


def _eq(a, b):
    return np.array_equal(a.cpu().numpy() if hasattr(a, "cpu") else a, b.cpu().numpy() if hasattr(b, "cpu") else b)


@pytest.mark.timeout(600)
def test_mid_workload_full_parity(db):
    print("mid workload: generating (k-mer counting on the GPU)", flush=True)
    w = synth.make_workload("mid", device="cuda:0")
    print(f"  reads {w.A.nrows} nnz(A) {w.A.nnz} nnz(R) {w.R.nnz}", flush=True)
    C = db.overlap(db.CSRTensors.from_numpy(w.A, "cuda:0"), w.min_shared)
    S, it = db.transitive_reduce(db.CSRTensors.from_numpy(w.R, "cuda:0"), w.fuzz)
    torch.cuda.synchronize()
    print("  oracle overlap ...", flush=True)
    ref = oracle.overlap(w.A, w.min_shared)
    assert _eq(C.rowptr, ref.rowptr) and _eq(C.col, ref.col)
    assert _eq(C.count, ref.count) and _eq(C.seed, ref.seed)
    print("  oracle reduction ...", flush=True)
    Sref, it_ref, _ = oracle.transitive_reduce(w.R, w.fuzz)
    assert it == it_ref
    assert _eq(S.rowptr, Sref.rowptr) and _eq(S.col, Sref.col) and _eq(S.val, Sref.val)


def _oracle_rows_threaded(A, min_shared, threads=16):
    """Every row of C = A A^T from the oracle, in row ranges balanced by
    products on `threads` threads that share one A^T (host memory: A^T once
    plus the ranges' outputs).  Returns (rowptr, col, count, seed)."""
    from concurrent.futures import ThreadPoolExecutor
    a = np.bincount(A.col, minlength=A.ncols).astype(np.int64)
    rp = np.add.reduceat(a[A.col], A.rowptr[:-1]) if A.nnz else np.zeros(A.nrows, np.int64)
    rp[np.diff(A.rowptr) == 0] = 0
    cs = np.cumsum(rp)
    cuts = [0] + [int(np.searchsorted(cs, cs[-1] * q / threads)) for q in range(1, threads)] + [A.nrows]
    at = oracle.transpose(A)
    ranges = [(cuts[q], cuts[q + 1]) for q in range(threads) if cuts[q + 1] > cuts[q]]
    with ThreadPoolExecutor(len(ranges)) as ex:
        parts = list(ex.map(lambda r: oracle.overlap(A, min_shared, rows=np.arange(r[0], r[1]), at=at), ranges))
    del at
    lens = np.concatenate([np.diff(p.rowptr) for p in parts])
    rowptr = np.concatenate([[0], np.cumsum(lens)])
    return (rowptr, np.concatenate([p.col for p in parts]), np.concatenate([p.count for p in parts]),
            np.concatenate([p.seed for p in parts]))


@pytest.mark.timeout(1100)
def test_large_workload_full_parity(db):
    """One GPU's share of the large run at full size: the GPU computes all of
    C and the reduction to its fixed point; the oracle recomputes every row
    of C (row ranges on 16 threads sharing one A^T) and the whole
    reduction."""
    print("large workload: generating (k-mer counting on the GPU)", flush=True)
    w = synth.make_workload("large", device="cuda:0")
    A, R = w.A, w.R
    print(f"  reads {A.nrows} kmers {A.ncols} nnz(A) {A.nnz} nnz(R) {R.nnz}", flush=True)
    Ad = db.CSRTensors.from_numpy(A, "cuda:0")
    C = db.overlap(Ad, w.min_shared)
    st = db.last_stats()
    print(f"  GPU overlap: nnz(C) {C.nnz}, products {st['products']}", flush=True)
    # the blocked overlap graph (4 blocks of reads, A^T over 4 column ranges
    # of slices, three-level sorts per range) equals R from the seeds of this
    # C, which the oracle checks in full below (A's values are positions here,
    # so the strand bit R from seeds reads is the position's low bit: the
    # same input for both builds)
    lens = torch.as_tensor(np.diff(w.reads.offsets).astype(np.int32), device="cuda:0")
    Rw = db.r_from_seeds(C, lens, w.k, 1000, 150, 52)
    Rb, nb = db.overlap_graph_blocked(Ad, w.min_shared, lens, w.k, 1000, 150, 52, block_rows=-(-A.nrows // 4))
    torch.cuda.synchronize()
    print(f"  blocked overlap graph: {nb} blocks, nnz(R) {Rb.nnz} (whole {Rw.nnz})", flush=True)
    assert nb == 4 and Rw.nnz > 0
    assert all(torch.equal(x, y) for x, y in ((Rb.rowptr, Rw.rowptr), (Rb.col, Rw.col), (Rb.val, Rw.val)))
    del Rw, Rb, Ad
    S, it = db.transitive_reduce(db.CSRTensors.from_numpy(R, "cuda:0"), w.fuzz)
    torch.cuda.synchronize()
    print(f"  GPU reduction: nnz(S) {S.nnz}, passes {it}", flush=True)
    assert st["products"] == synth.overlap_products(A)
    rowptr, col, cnt = C.rowptr.cpu().numpy(), C.col.cpu().numpy(), C.count.cpu().numpy()
    seed = C.seed.cpu().numpy().reshape(-1, 4)
    del C
    print("  oracle overlap, all rows on 16 threads ...", flush=True)
    ref = _oracle_rows_threaded(A, w.min_shared)
    assert np.array_equal(rowptr, ref[0])
    assert np.array_equal(col, ref[1]) and np.array_equal(cnt, ref[2]) and np.array_equal(seed, ref[3])
    del ref, col, cnt, seed
    print("  oracle reduction ...", flush=True)
    Sref, it_ref, _ = oracle.transitive_reduce(R, w.fuzz)
    assert it == it_ref
    assert _eq(S.rowptr, Sref.rowptr) and _eq(S.col, Sref.col) and _eq(S.val, Sref.val)


@pytest.mark.timeout(600)
def test_mid_workload_hash_path_full_parity(db):
    """The mid-size workload through the LDS-hash symbolic and numeric path
    (no bitmap), including the retry table for rows that overflow the first
    table, against the oracle in full."""
    w = synth.make_workload("mid", device="cuda:0")
    A = db.CSRTensors.from_numpy(w.A, "cuda:0")
    old = db.get_tuning()
    try:
        db.set_tuning(bits_max_words=0)
        C = db.overlap(A, w.min_shared)
        # a small first table sends many rows to the retry level
        db.set_tuning(bits_max_words=0, sym_first_log2=9)
        C2 = db.overlap(A, w.min_shared)
        torch.cuda.synchronize()
    finally:
        db.set_tuning(**old)
    print(f"  nnz(C) {C.nnz}; oracle ...", flush=True)
    ref = oracle.overlap(w.A, w.min_shared)
    for X in (C, C2):
        assert _eq(X.rowptr, ref.rowptr) and _eq(X.col, ref.col)
        assert _eq(X.count, ref.count) and _eq(X.seed, ref.seed)


@pytest.mark.timeout(900)
def test_batchset_workload_full_parity(db):
    """The batching workload at full size (64 uneven read sets in one batched
    overlap call and one batched, graph-captured reduction call) against the
    oracle, set by set."""
    print("batching workload: generating 64 sets", flush=True)
    ws = synth.batch_workloads(64, device="cuda:0")
    As = [db.CSRTensors.from_numpy(w.A, "cuda:0") for w in ws]
    Rs = [db.CSRTensors.from_numpy(w.R, "cuda:0") for w in ws]
    Cs = db.overlap_batched(As, [w.min_shared for w in ws])
    Ss, its = db.transitive_reduce_batched(Rs, [w.fuzz for w in ws], graph=True)
    torch.cuda.synchronize()
    print(f"  reads {sum(w.A.nrows for w in ws)}, products {sum(synth.overlap_products(w.A) for w in ws)}; "
          "oracle ...", flush=True)
    for s, w in enumerate(ws):
        ref = oracle.overlap(w.A, w.min_shared)
        C = Cs[s]
        assert _eq(C.rowptr, ref.rowptr) and _eq(C.col, ref.col), s
        assert _eq(C.count, ref.count) and _eq(C.seed, ref.seed), s
        Sref, it_ref, _ = oracle.transitive_reduce(w.R, w.fuzz)
        assert its[s] == it_ref, s
        assert _eq(Ss[s].rowptr, Sref.rowptr) and _eq(Ss[s].col, Sref.col) and _eq(Ss[s].val, Sref.val), s


def test_serve_mix_equals_solo_and_oracle(db):
    """Continuous batching over four slots (threads with their own streams):
    every job's C, R (from C's seeds) and S in the mix equal the same job run
    alone (tolerance 0), and equal the oracle's C, R from the oracle's C and
    S from the oracle's R."""
    from paper_2010_10055_amd import serve
    pool = serve.make_pool([("tiny", 3, 7000, 1.0), ("batchset", 3, 7100, 0.05)], device="cuda:0",
                           keep_host=True)
    rng = np.random.default_rng(5)
    jobs = serve.draw_jobs(rng, pool, 24, rate=2000.0, small_fraction=0.5)
    clock = serve.WallClock()
    ex = serve.GpuSlots(4, clock, keep_results=True)
    st = {}
    try:
        done = serve.serve(jobs, ex, clock, hbm_budget=serve.hbm_free_bytes(), slots=4, stats=st)
    finally:
        ex.close()
    assert len(done) == 24 and all(d.error is None for d in done), [d.error for d in done if d.error]
    assert st["peak_running"] > 1
    by = {d.jid: d for d in done}
    refs = {}
    for j in jobs:
        C1, R1, S1, it1 = by[j.jid].result
        C0, R0, S0, it0 = serve.run_layout(j.payload)
        torch.cuda.synchronize()
        assert it1 == it0
        for f in ("rowptr", "col", "count", "seed"):
            assert torch.equal(getattr(C1, f), getattr(C0, f)), (j.jid, "C", f)
        for X1, X0, tag in ((R1, R0, "R"), (S1, S0, "S")):
            for f in ("rowptr", "col", "val"):
                assert torch.equal(getattr(X1, f), getattr(X0, f)), (j.jid, tag, f)
        inp = j.payload
        if id(inp) not in refs:
            Cref = oracle.overlap(inp.host_A, inp.min_shared)
            Rref = oracle.r_from_seeds(Cref, inp.host_len, inp.k, inp.min_overlap, inp.max_drift, inp.min_density)
            Sref, itref, _ = oracle.transitive_reduce(Rref, inp.fuzz)
            refs[id(inp)] = (Cref, Rref, Sref, itref)
        Cref, Rref, Sref, itref = refs[id(inp)]
        assert _eq(C1.rowptr, Cref.rowptr) and _eq(C1.col, Cref.col), j.jid
        assert _eq(C1.count, Cref.count) and _eq(C1.seed, Cref.seed), j.jid
        assert _eq(R1.rowptr, Rref.rowptr) and _eq(R1.col, Rref.col) and _eq(R1.val, Rref.val), j.jid
        assert it1 == itref
        assert _eq(S1.rowptr, Sref.rowptr) and _eq(S1.col, Sref.col) and _eq(S1.val, Sref.val), j.jid


def test_autotuned_configuration_keeps_bits(db, tmp_path):
    """The tuner keeps only candidates whose outputs equal the starting
    configuration's element by element; the tuned configuration reproduces
    them and the oracle's."""
    from paper_2010_10055_amd import autotune
    ws = [synth.make_workload("tiny", seed=1000 + s) for s in range(4)]
    As = [db.CSRTensors.from_numpy(w.A, "cuda:0") for w in ws]
    Rs = [db.CSRTensors.from_numpy(w.R, "cuda:0") for w in ws]
    old = db.get_tuning()
    try:
        def run():
            Cs = db.overlap_batched(As, 1)
            Ss, its = db.transitive_reduce_batched(Rs, 1000, graph=True)
            return Cs, Ss, its

        ref = autotune.snapshot(run())
        cfg = autotune.autotune(run, "test-key", budget_s=20, repeats=1, cache_file=str(tmp_path / "c.json"),
                                force=True, log=lambda s: None)
        assert db.get_tuning() == cfg
        res = run()
        torch.cuda.synchronize()
        assert autotune.results_equal(ref, res)
        Cs, Ss, its = res
        for s, w in enumerate(ws):
            ref_c = oracle.overlap(w.A, 1)
            assert _eq(Cs[s].col, ref_c.col) and _eq(Cs[s].seed, ref_c.seed) and _eq(Cs[s].count, ref_c.count)
            Sref, it_ref, _ = oracle.transitive_reduce(w.R, 1000)
            assert its[s] == it_ref and _eq(Ss[s].val, Sref.val)
        assert autotune.load_cache(str(tmp_path / "c.json"))["test-key"]["tuning"] == cfg
    finally:
        db.set_tuning(**old)


def test_batched_graph_and_plain_reductions_agree(db):
    ws = synth.batch_workloads(6, seed=4100, scale=0.05)
    Rs = [db.CSRTensors.from_numpy(w.R, "cuda:0") for w in ws]
    S0, it0 = db.transitive_reduce_batched(Rs, 1000, graph=False)
    S1, it1 = db.transitive_reduce_batched(Rs, 1000, graph=True)
    assert it0 == it1
    for s, w in enumerate(ws):
        ref, it_ref, _ = oracle.transitive_reduce(w.R, 1000)
        assert it0[s] == it_ref
        assert _eq(S0[s].col, ref.col) and _eq(S1[s].val, ref.val)
