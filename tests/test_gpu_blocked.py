"""GPU parity of the blocked overlap graph (dibella_overlap_graph_blocked:
C formed a block of reads at a time, turned into R and released) against
the oracle's R from the seeds of the whole C, bit for bit, for block sizes
from one read to more than all of them; the hash path and the sliced
segment pass run blocked too."""
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


def _eq(t, a):
    return np.array_equal(t.cpu().numpy(), a)


def _lens(reads, dev="cuda:0"):
    return torch.as_tensor(np.diff(reads.offsets).astype(np.int32), device=dev)


def _oracle_r(w, min_overlap, drift, density):
    C = oracle.overlap(w.A, w.min_shared)
    return oracle.r_from_seeds(C, np.diff(w.reads.offsets), w.k, min_overlap, drift, density)


@pytest.fixture(scope="module")
def tiny():
    return synth.make_workload("tiny", strand_bit=True)


@pytest.mark.parametrize("block_rows", [1, 7, 64, 199, 200, 1 << 20])
def test_blocked_graph_matches_oracle(db, tiny, block_rows):
    w = tiny
    print(f"tiny: reads {w.A.nrows}, block_rows {block_rows}", flush=True)
    ref = _oracle_r(w, 200, 150, 16)
    R, nb = db.overlap_graph_blocked(db.CSRTensors.from_numpy(w.A, "cuda:0"), w.min_shared, _lens(w.reads), w.k,
                                     200, 150, 16, block_rows=block_rows)
    torch.cuda.synchronize()
    assert nb == -(-w.A.nrows // block_rows)
    assert R.nrows == R.ncols == w.A.nrows
    assert _eq(R.rowptr, ref.rowptr) and _eq(R.col, ref.col) and _eq(R.val, ref.val)


def test_blocked_graph_equals_unblocked_library_path(db):
    """A batch-sized workload (ragged last block), without the drift and
    density tests: the blocked R equals r_from_seeds of the library's whole C
    and the oracle's."""
    w = synth.make_workload("batchset", strand_bit=True, seed=4011)
    print(f"batchset: reads {w.A.nrows} nnz(A) {w.A.nnz}", flush=True)
    A = db.CSRTensors.from_numpy(w.A, "cuda:0")
    L = _lens(w.reads)
    whole = db.r_from_seeds(db.overlap(A, w.min_shared), L, w.k, 1000)
    ref = _oracle_r(w, 1000, -1, 0)
    for block_rows in (max(1, w.A.nrows // 3), w.A.nrows // 3 + 1):
        R, nb = db.overlap_graph_blocked(A, w.min_shared, L, w.k, 1000, block_rows=block_rows)
        torch.cuda.synchronize()
        assert nb >= 3
        for a, b in ((R.rowptr, whole.rowptr), (R.col, whole.col), (R.val, whole.val)):
            assert torch.equal(a, b)
        assert _eq(R.rowptr, ref.rowptr) and _eq(R.col, ref.col) and _eq(R.val, ref.val)


def test_blocked_graph_hash_path(db, tiny):
    """With the bitmap path switched off every block's rows take the LDS
    hash tables (and their retry level)."""
    w = tiny
    t0 = db.get_tuning()
    try:
        db.set_tuning(bits_max_words=0)
        R, nb = db.overlap_graph_blocked(db.CSRTensors.from_numpy(w.A, "cuda:0"), w.min_shared, _lens(w.reads),
                                         w.k, 200, -1, 0, block_rows=50)
        torch.cuda.synchronize()
    finally:
        db.set_tuning(**t0)
    ref = _oracle_r(w, 200, -1, 0)
    assert nb == 4
    assert _eq(R.rowptr, ref.rowptr) and _eq(R.col, ref.col) and _eq(R.val, ref.val)


@pytest.mark.timeout(900)
def test_blocked_graph_mid_workload_sliced(db):
    """The mid-size workload: enough columns for the sliced segment pass, so
    every block reads its rows' part of the slice table, and A^T is built
    over as many column ranges of slices as there are blocks (5 ranges for
    blocks of 7000 reads; 8, every slice, for blocks of 600).  Both against
    the oracle's R from the whole C."""
    w = synth.make_workload("mid", device="cuda:0", strand_bit=True)
    print(f"mid: reads {w.A.nrows} nnz(A) {w.A.nnz} k-mers {w.A.ncols}", flush=True)
    A = db.CSRTensors.from_numpy(w.A, "cuda:0")
    got = {}
    for block_rows in (7000, 600):
        R, nb = db.overlap_graph_blocked(A, w.min_shared, _lens(w.reads), w.k, 1000, 100, 16, block_rows=block_rows)
        torch.cuda.synchronize()
        assert nb == -(-w.A.nrows // block_rows)
        got[block_rows] = (R.rowptr.cpu().numpy(), R.col.cpu().numpy(), R.val.cpu().numpy())
        print(f"  blocks of {block_rows}: {nb} blocks, nnz(R) {R.nnz}", flush=True)
    print("  oracle ...", flush=True)
    ref = _oracle_r(w, 1000, 100, 16)
    for rp, col, val in got.values():
        assert np.array_equal(rp, ref.rowptr) and np.array_equal(col, ref.col) and np.array_equal(val, ref.val)


def test_blocked_graph_argument_errors(db, tiny):
    w = tiny
    A = db.CSRTensors.from_numpy(w.A, "cuda:0")
    L = _lens(w.reads)
    with pytest.raises(db.DibellaError):
        db.overlap_graph_blocked(A, w.min_shared, L, w.k, 200, block_rows=0)
    with pytest.raises(db.DibellaError):
        db.overlap_graph_blocked(A, w.min_shared, L, 0, 200, block_rows=10)
    with pytest.raises(db.DibellaError):
        db.overlap_graph_blocked(A, 0, L, w.k, 200, block_rows=10)
    # a malformed A fails before any block: an unsorted row
    col = w.A.col.copy()
    lo = int(w.A.rowptr[3])
    col[lo], col[lo + 1] = col[lo + 1], col[lo]
    bad = db.CSRTensors(w.A.nrows, w.A.ncols, torch.as_tensor(w.A.rowptr, device="cuda:0"),
                        torch.as_tensor(col, device="cuda:0"), torch.as_tensor(w.A.val, device="cuda:0"))
    with pytest.raises(db.DibellaError):
        db.overlap_graph_blocked(bad, w.min_shared, L, w.k, 200, block_rows=10)
    # the library still works afterwards
    R, _ = db.overlap_graph_blocked(A, w.min_shared, L, w.k, 200, block_rows=10)
    ref = _oracle_r(w, 200, -1, 0)
    assert _eq(R.col, ref.col) and _eq(R.val, ref.val)
