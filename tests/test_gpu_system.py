"""GPU system tests: the mid-size workload against the oracle at full size,
the large workload at full size against the oracle on sampled rows of C and
on the whole reduction, the batching workload (64 sets) in full,
the serving loop (each job's result in the mix equals its solo result,
tolerance 0), the autotuner (tuned configurations reproduce the default
bits), and batched graph-captured reductions."""
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


@pytest.mark.timeout(900)
def test_large_workload_sampled_parity(db):
    """One GPU's share of the large run at full size: the GPU computes all of
    C and the reduction to its fixed point; the oracle recomputes a sample of
    C's rows (random rows, the longest rows, the first and last) and the whole
    reduction."""
    print("large workload: generating (k-mer counting on the GPU)", flush=True)
    w = synth.make_workload("large", device="cuda:0")
    A, R = w.A, w.R
    print(f"  reads {A.nrows} kmers {A.ncols} nnz(A) {A.nnz} nnz(R) {R.nnz}", flush=True)
    C = db.overlap(db.CSRTensors.from_numpy(A, "cuda:0"), w.min_shared)
    st = db.last_stats()
    print(f"  GPU overlap: nnz(C) {C.nnz}, products {st['products']}", flush=True)
    S, it = db.transitive_reduce(db.CSRTensors.from_numpy(R, "cuda:0"), w.fuzz)
    torch.cuda.synchronize()
    print(f"  GPU reduction: nnz(S) {S.nnz}, passes {it}", flush=True)
    assert st["products"] == synth.overlap_products(A)
    rng = np.random.default_rng(31)
    lens = np.diff(A.rowptr)
    rows = np.unique(np.concatenate([rng.choice(A.nrows, 300, replace=False), np.argsort(lens)[-8:],
                                     [0, A.nrows - 1]])).astype(np.int64)
    print(f"  oracle overlap on {rows.size} rows ...", flush=True)
    ref = oracle.overlap(A, w.min_shared, rows=rows)
    rp = C.rowptr.cpu().numpy()
    col, cnt, seed = C.col.cpu().numpy(), C.count.cpu().numpy(), C.seed.cpu().numpy().reshape(-1, 4)
    for q, i in enumerate(rows):
        a, b = rp[i], rp[i + 1]
        x, y = ref.rowptr[q], ref.rowptr[q + 1]
        assert b - a == y - x, f"row {i}: {b - a} entries vs {y - x}"
        assert np.array_equal(col[a:b], ref.col[x:y]), f"row {i} col"
        assert np.array_equal(cnt[a:b], ref.count[x:y]), f"row {i} count"
        assert np.array_equal(seed[a:b], ref.seed[x:y]), f"row {i} seed"
    print("  oracle reduction ...", flush=True)
    Sref, it_ref, _ = oracle.transitive_reduce(R, w.fuzz)
    assert it == it_ref
    assert _eq(S.rowptr, Sref.rowptr) and _eq(S.col, Sref.col) and _eq(S.val, Sref.val)


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


def test_serve_mix_equals_solo(db):
    from paper_2010_10055_amd import serve
    pool = serve.make_pool([("tiny", 3, 7000, 1.0), ("batchset", 3, 7100, 0.05)], device="cuda:0")
    rng = np.random.default_rng(5)
    jobs = serve.draw_jobs(rng, pool, 24, rate=2000.0, small_fraction=0.5)
    clock = serve.WallClock()
    done = serve.serve(jobs, serve.gpu_executor(batched=True), clock, hbm_budget=8 << 30, max_batch=16)
    assert len(done) == 24 and all(d.error is None for d in done)
    assert max(sum(1 for d in done if d.batch == b) for b in {d.batch for d in done}) > 1
    solo = serve.gpu_executor(batched=False)
    by = {d.jid: d for d in done}
    for j in jobs:
        C1, S1, it1 = by[j.jid].result
        C0, S0, it0 = solo([j])[0]
        assert it1 == it0
        for f in ("rowptr", "col", "count", "seed"):
            assert torch.equal(getattr(C1, f), getattr(C0, f)), (j.jid, f)
        for f in ("rowptr", "col", "val"):
            assert torch.equal(getattr(S1, f), getattr(S0, f)), (j.jid, f)


def test_autotuned_configuration_keeps_bits(db, tmp_path):
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

        def fp(res):
            Cs, Ss, its = res
            return (tuple(int(c.col.sum()) for c in Cs), tuple(int(c.seed.sum()) for c in Cs),
                    tuple(int(s.val.sum()) for s in Ss), tuple(its))

        ref = fp(run())
        cfg = autotune.autotune(run, fp, "test-key", budget_s=20, repeats=1, cache_file=str(tmp_path / "c.json"),
                                force=True, log=lambda s: None)
        assert db.get_tuning() == cfg
        Cs, Ss, its = run()
        for s, w in enumerate(ws):
            ref_c = oracle.overlap(w.A, 1)
            assert _eq(Cs[s].col, ref_c.col) and _eq(Cs[s].seed, ref_c.seed)
        assert fp((Cs, Ss, its)) == ref
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
