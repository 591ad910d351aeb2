"""GPU parity of A from the reads (dibella_kmer_matrix: windows, canonical
k-mers, frequencies, reliable columns, smallest positions) against the
oracle, bit for bit, on the tiny and batch workloads and on hand-made read
sets (short and empty reads, palindromes, k = 1 to 31, bounds); the mid
and large workloads against the generator's A (torch), which the CPU tests
check equal to the oracle's on the tiny workload."""
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


def _dev(bases, offsets):
    return (torch.as_tensor(np.ascontiguousarray(bases, dtype=np.uint8), device="cuda:0"),
            torch.as_tensor(np.ascontiguousarray(offsets, dtype=np.int64), device="cuda:0"))


def _check(db, bases, offsets, k, lo, hi, strand):
    A, codes = db.kmer_matrix(*_dev(bases, offsets), k, lo, hi, strand)
    ref, ref_codes = oracle.kmer_matrix(bases, offsets, k, lo, hi, strand)
    torch.cuda.synchronize()
    assert A.nrows == ref.nrows and A.ncols == ref.ncols
    assert np.array_equal(A.rowptr.cpu().numpy(), ref.rowptr)
    assert np.array_equal(A.col.cpu().numpy(), ref.col)
    assert np.array_equal(A.val.cpu().numpy(), ref.val)
    assert np.array_equal(codes.cpu().numpy().astype(np.uint64), ref_codes)
    return A


@pytest.fixture(scope="module")
def tiny():
    return synth.make_workload("tiny")


@pytest.mark.parametrize("k,lo,hi,strand", [(17, 2, 8, False), (17, 2, 8, True), (5, 2, 40, True),
                                            (31, 1, 3, True), (11, 1, 1, False), (17, 3, 1000, True)])
def test_kmer_matrix_tiny_matches_oracle(db, tiny, k, lo, hi, strand):
    print(f"tiny: k {k} bounds [{lo}, {hi}] strand {strand}", flush=True)
    A = _check(db, tiny.reads.bases, tiny.reads.offsets, k, lo, hi, strand)
    if (k, lo, hi, strand) == (17, 2, 8, False):
        assert A.nnz == tiny.A.nnz   # the workload's own A


@pytest.mark.parametrize("seed,k", [(0, 1), (1, 2), (2, 4), (3, 5), (4, 9)])
def test_kmer_matrix_small_reads_matches_oracle(db, seed, k):
    """Reads of 0 to 40 bases (many without a window), a repeat, even k with
    palindromic k-mers, k = 1."""
    rng = np.random.default_rng(700 + seed)
    lens = rng.integers(0, 41, size=60)
    lens[:3] = [0, k - 1, k]
    g = rng.integers(0, 4, size=int(lens.sum()), dtype=np.uint8)
    g[200:230] = g[10:40]
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    print(f"small reads: seed {seed} k {k} bases {len(g)}", flush=True)
    for lo, hi, strand in ((1, 1000, True), (2, 5, False)):
        _check(db, g, off, k, lo, hi, strand)


def test_kmer_matrix_no_reads_and_no_windows(db):
    A, codes = db.kmer_matrix(*_dev(np.zeros(0, np.uint8), np.zeros(1, np.int64)), 17, 1, 10)
    assert A.nrows == 0 and A.ncols == 0 and A.nnz == 0 and codes.numel() == 0
    A, codes = _check(db, np.array([1, 2, 3], np.uint8), np.array([0, 3, 3], np.int64), 5, 1, 10, True), None
    assert A.nrows == 2 and A.nnz == 0 and A.rowptr.cpu().tolist() == [0, 0, 0]


def test_kmer_matrix_batchset_matches_oracle(db):
    w = synth.make_workload("batchset", seed=4021)
    print(f"batchset: reads {w.reads.n} bases {len(w.reads.bases)}", flush=True)
    _check(db, w.reads.bases, w.reads.offsets, w.k, w.lo, w.hi, True)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name", ["mid", "large"])
def test_kmer_matrix_equals_the_generator(db, name):
    """At the mid and large sizes the oracle's sort of every window is too
    slow for a test: the library's A (strand bits) against the generator's."""
    w = synth.make_workload(name, device="cuda:0", strand_bit=True)
    print(f"{name}: reads {w.reads.n} bases {len(w.reads.bases)} nnz(A) {w.A.nnz}", flush=True)
    A, codes = db.kmer_matrix(*_dev(w.reads.bases, w.reads.offsets), w.k, w.lo, w.hi, True)
    torch.cuda.synchronize()
    assert A.ncols == w.A.ncols and A.nnz == w.A.nnz
    assert np.array_equal(A.rowptr.cpu().numpy(), w.A.rowptr)
    assert np.array_equal(A.col.cpu().numpy(), w.A.col)
    assert np.array_equal(A.val.cpu().numpy(), w.A.val)


def test_kmer_matrix_argument_errors(db):
    b, o = _dev(np.array([0, 1, 2, 3, 0, 1], np.uint8), np.array([0, 6], np.int64))
    for k, lo, hi in ((0, 1, 2), (32, 1, 2), (3, 0, 2), (3, 3, 2)):
        with pytest.raises(db.DibellaError):
            db.kmer_matrix(b, o, k, lo, hi)
    with pytest.raises(db.DibellaError):   # a base outside 0..3
        db.kmer_matrix(*_dev(np.array([0, 1, 4, 3, 0, 1], np.uint8), np.array([0, 6], np.int64)), 3, 1, 5)
    with pytest.raises(db.DibellaError):   # offsets that go back
        db.kmer_matrix(*_dev(np.array([0, 1, 2, 3, 0, 1], np.uint8), np.array([0, 4, 2, 6], np.int64)), 3, 1, 5)
    with pytest.raises(db.DibellaError):   # offsets that do not end at the bases' end
        db.kmer_matrix(*_dev(np.array([0, 1, 2, 3, 0, 1], np.uint8), np.array([0, 5], np.int64)), 3, 1, 5)
    A, _ = db.kmer_matrix(b, o, 3, 1, 5)   # still works
    assert A.nnz > 0
