"""Pins for the CPU oracle (no GPU).

The oracle is checked against things it does not contain itself:
brute force from the raw read strings, scipy's sparse product, closed forms
for the diagonal and the total count, the paper's worked example, networkx's
transitive reduction of DAGs, and the exact string graph of error-free reads.
"""
import json
import types
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_2010_10055_amd import synth
from tests import bruteforce

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _small_reads_workload(seed, G=30_000, n_reads=40, err=0.15, fams=(), lo=2, hi=8):
    rng = np.random.default_rng(seed)
    g = synth.insert_repeats(rng, synth.random_genome(rng, G), list(fams))
    reads = synth.sample_reads(rng, g, n_reads=n_reads, length_uniform=(1000, 4000),
                               error_rate=err)
    A, _ = synth.kmer_matrix(reads, 17, lo, hi)
    return reads, A


def _c_as_dict(C):
    out = {}
    for i in range(C.nrows):
        for e in range(int(C.rowptr[i]), int(C.rowptr[i + 1])):
            out[(i, int(C.col[e]))] = (int(C.count[e]), tuple(int(x) for x in C.seed[e]))
    return out


# ---------------------------------------------------------------------------
# Overlap  C = A A^T
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed,min_shared,fams,lo,hi", [
    (11, 1, (), 2, 8),
    (12, 2, ((500, 6, 0.01),), 2, 8),
    (13, 3, ((300, 12, 0.02),), 2, 20),
])
def test_overlap_equals_bruteforce_from_reads(seed, min_shared, fams, lo, hi):
    reads, A = _small_reads_workload(seed, fams=fams, lo=lo, hi=hi)
    expect, n_reliable = bruteforce.overlap_from_reads(reads, 17, lo, hi, min_shared)
    assert A.ncols == n_reliable
    C = oracle.overlap(A, min_shared)
    assert _c_as_dict(C) == expect


def test_overlap_tiny_workload_bruteforce():
    w = synth.make_workload("tiny")
    expect, _ = bruteforce.overlap_from_reads(w.reads, 17, w.lo, w.hi, w.min_shared)
    C = oracle.overlap(w.A, w.min_shared)
    got = _c_as_dict(C)
    assert len(got) == len(expect)
    assert got == expect


def _pattern(A):
    return sp.csr_matrix((np.ones(A.nnz, np.int64), A.col, A.rowptr), shape=(A.nrows, A.ncols))


@pytest.mark.parametrize("seed,n,m,density,min_shared", [
    (1, 60, 300, 0.05, 1), (2, 80, 200, 0.1, 2), (3, 50, 1000, 0.01, 1), (4, 1, 10, 0.5, 1),
])
def test_overlap_counts_equal_scipy_product(seed, n, m, density, min_shared):
    rng = np.random.default_rng(seed)
    A = synth.random_a(rng, n, m, density)
    C = oracle.overlap(A, min_shared)
    P = _pattern(A)
    ref = (P @ P.T).tocsr()
    ref.data[ref.data < min_shared] = 0
    ref.eliminate_zeros()
    ref.sort_indices()
    assert np.array_equal(C.rowptr, ref.indptr.astype(np.int64))
    assert np.array_equal(C.col, ref.indices.astype(np.int32))
    assert np.array_equal(C.count, ref.data.astype(np.int32))


def test_overlap_invariants_on_tiny_workload():
    w = synth.make_workload("tiny")
    A = w.A
    C = oracle.overlap(A, 1)
    d = _c_as_dict(C)
    # symmetry with each seed pair swapped
    for (i, j), (c, s) in d.items():
        assert d[(j, i)] == (c, (s[1], s[0], s[3], s[2]))
    # diagonal closed form: count = nnz(A_i); seeds = first two positions twice
    for i in range(A.nrows):
        cols, vals = A.row(i)
        if cols.size == 0:
            assert (i, i) not in d
            continue
        s1 = (int(vals[1]), int(vals[1])) if cols.size > 1 else (-1, -1)
        assert d[(i, i)] == (cols.size, (int(vals[0]), int(vals[0])) + s1)
    # total count = sum over k-mers of (column count)^2
    assert int(C.count.astype(np.int64).sum()) == synth.overlap_products(A)


def test_overlap_seeds_smallest_two_kmers_adversarial():
    # one column shared by every row plus a dense row
    rng = np.random.default_rng(7)
    A = synth.random_a(rng, 40, 120, 0.05, dense_rows=[3], dense_cols=[0, 57])
    C = oracle.overlap(A, 1)
    d = _c_as_dict(C)
    for (i, j), (c, s) in d.items():
        ci, vi = A.row(i)
        cj, vj = A.row(j)
        shared = sorted(set(ci.tolist()) & set(cj.tolist()))
        assert c == len(shared)
        k0 = shared[0]
        exp = [int(vi[ci == k0][0]), int(vj[cj == k0][0]), -1, -1]
        if len(shared) > 1:
            k1 = shared[1]
            exp[2:] = [int(vi[ci == k1][0]), int(vj[cj == k1][0])]
        assert s == tuple(exp)


def test_overlap_row_subset_matches_full():
    w = synth.make_workload("tiny")
    full = oracle.overlap(w.A, 1)
    rows = np.array([5, 0, 199, 77, 77])
    sub = oracle.overlap(w.A, 1, rows=rows)
    for r, i in enumerate(rows):
        a, b = full.rowptr[i], full.rowptr[i + 1]
        c, d = sub.rowptr[r], sub.rowptr[r + 1]
        assert np.array_equal(full.col[a:b], sub.col[c:d])
        assert np.array_equal(full.count[a:b], sub.count[c:d])
        assert np.array_equal(full.seed[a:b], sub.seed[c:d])


def test_transpose_lists_each_column_by_read():
    """A^T built once: row k lists (read, position) of every A entry in column
    k, reads increasing (checked against a direct scipy transpose)."""
    rng = np.random.default_rng(41)
    A = synth.random_a(rng, 120, 400, 0.03)
    at = oracle.transpose(A)
    n = A.nrows
    rows = np.repeat(np.arange(n), np.diff(A.rowptr))
    T = sp.csr_matrix((A.val.astype(np.int64) + 1, (A.col, rows)), shape=(A.ncols, n))
    T.sort_indices()
    assert np.array_equal(at.rowptr, T.indptr)
    assert np.array_equal(at.read, T.indices)
    assert np.array_equal(at.pos.astype(np.int64), T.data - 1)


def test_overlap_with_shared_transpose_in_row_ranges():
    """Row ranges computed with one shared A^T (as threads do) concatenate to
    the full product."""
    w = synth.make_workload("tiny")
    full = oracle.overlap(w.A, 1)
    at = oracle.transpose(w.A)
    cuts = [0, 37, 38, 120, w.A.nrows]
    parts = [oracle.overlap(w.A, 1, rows=np.arange(a, b), at=at) for a, b in zip(cuts[:-1], cuts[1:])]
    assert np.array_equal(np.concatenate([p.col for p in parts]), full.col)
    assert np.array_equal(np.concatenate([p.count for p in parts]), full.count)
    assert np.array_equal(np.concatenate([p.seed for p in parts]), full.seed)
    lens = np.concatenate([np.diff(p.rowptr) for p in parts])
    assert np.array_equal(lens, np.diff(full.rowptr))


def test_overlap_empty_inputs():
    A = synth.CSR(3, 5, np.zeros(4, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32))
    C = oracle.overlap(A, 1)
    assert C.col.size == 0 and np.all(C.rowptr == 0)
    A0 = synth.CSR(0, 0, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32))
    C0 = oracle.overlap(A0, 1)
    assert C0.rowptr.size == 1


# ---------------------------------------------------------------------------
# Transitive reduction
# ---------------------------------------------------------------------------

def _dense_to_r(values, codes=None):
    n = len(values)
    rows, cols, vals = [], [], []
    for i in range(n):
        for j in range(n):
            if values[i][j]:
                c = 0 if codes is None else codes[i][j]
                rows.append(i)
                cols.append(j)
                vals.append((values[i][j] << 2) | c)
    return synth.coo_to_csr(n, n, rows, cols, vals)


def _s_dense(S):
    D = np.zeros((S.nrows, S.nrows), np.int64)
    for i in range(S.nrows):
        for e in range(int(S.rowptr[i]), int(S.rowptr[i + 1])):
            D[i, int(S.col[e])] = int(S.val[e]) >> 2
    return D


def test_worked_example_from_paper():
    g = json.load(open(os.path.join(GOLDEN, "tr_worked_example.json")))
    R = _dense_to_r(g["R"])
    for rule in ("row", "edge"):
        for variant in ("A", "B"):
            S, iters, trace = oracle.transitive_reduce(R, g["x"], variant, rule)
            assert _s_dense(S).tolist() == g["S"]
            assert iters == g["productive_passes"] + 1
    marks = oracle.tr_pass_marks(R, g["x"])
    got_I = np.zeros((4, 4), np.int64)
    for i in range(4):
        for e in range(int(R.rowptr[i]), int(R.rowptr[i + 1])):
            got_I[i, R.col[e]] = marks[e]
    assert got_I.tolist() == g["I"]
    # N, v and M of the example follow from R directly
    Rm = np.array(g["R"])
    for i in range(4):
        row = Rm[i][Rm[i] > 0]
        assert (row.max() if row.size else 0) == g["v"][i]
        for j in range(4):
            paths = [Rm[i][k] + Rm[k][j] for k in range(4) if Rm[i][k] and Rm[k][j]]
            assert (min(paths) if paths else 0) == g["N"][i][j]


@pytest.mark.parametrize("code", [(0, 0), (1, 1)])
def test_worked_example_uniform_orientation(code):
    g = json.load(open(os.path.join(GOLDEN, "tr_worked_example.json")))
    c = (code[0] << 1) | code[1]
    R = _dense_to_r(g["R"], [[c] * 4 for _ in range(4)])
    S, _, _ = oracle.transitive_reduce(R, g["x"])
    assert _s_dense(S).tolist() == g["S"]


def test_worked_example_invalid_walk_keeps_edge():
    # R_32 enters read 2 by one head and R_21 leaves by the same head:
    # 3 -> 2 -> 1 is not a valid walk, so 3 -> 1 stays (condition (a)).
    # 4 -> 3 -> 2 is still a valid walk but now ends with code (0, 1) while
    # R_42 has (0, 0): condition (c) fails and 4 -> 2 stays as well.
    g = json.load(open(os.path.join(GOLDEN, "tr_worked_example.json")))
    codes = [[0] * 4 for _ in range(4)]
    codes[2][1] = 0b01          # (o_src, o_dst) = (0, 1)
    R = _dense_to_r(g["R"], codes)
    S, _, _ = oracle.transitive_reduce(R, g["x"])
    D = _s_dense(S)
    assert D[2, 0] == 80 and D[3, 1] == 80


def test_worked_example_end_heads_must_match():
    # 3 -> 2 -> 1 is a valid walk with end code (0, 0), but R_31 has code
    # (0, 1): condition (c) fails, the edge stays.
    g = json.load(open(os.path.join(GOLDEN, "tr_worked_example.json")))
    codes = [[0] * 4 for _ in range(4)]
    codes[2][0] = 0b01
    R = _dense_to_r(g["R"], codes)
    S, _, _ = oracle.transitive_reduce(R, g["x"])
    assert _s_dense(S)[2, 0] == 80


@pytest.mark.parametrize("rule", ["row", "edge"])
def test_comparison_is_inclusive_at_equality(rule):
    # Triangle 0 -> 1 -> 2 with the chord 0 -> 2 (uniform orientation).  The
    # walk's overhang sum is a + b.  I = M >= N (Alg. TransitiveReduction):
    # the chord goes when a + b equals M exactly and stays when it is one
    # above.  M_02 = max overhang of row 0 + x (row rule) or R_02 + x (edge
    # rule).
    a, c, x = 300, 500, 1000
    M = (max(a, c) if rule == "row" else c) + x
    for b, gone in ((M - a, True), (M - a + 1, False)):
        R = _dense_to_r([[0, a, c], [0, 0, b], [0, 0, 0]])
        S, _, _ = oracle.transitive_reduce(R, x, "A", rule)
        assert (_s_dense(S)[0, 2] == 0) == gone, (rule, b)
        marks = oracle.tr_pass_marks(R, x, "A", rule)
        assert bool(marks[1]) == gone     # row 0 holds (0,1) then (0,2)


def _dense_from_bf(D, n):
    out = np.zeros((n, n), np.int64) - 1
    for i in range(n):
        for j in range(n):
            if D[i][j] is not None:
                out[i, j] = D[i][j]
    return out


def _s_packed(S):
    out = np.zeros((S.nrows, S.nrows), np.int64) - 1
    for i in range(S.nrows):
        for e in range(int(S.rowptr[i]), int(S.rowptr[i + 1])):
            out[i, int(S.col[e])] = int(S.val[e])
    return out


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("variant,rule", [("A", "row"), ("B", "row"), ("A", "edge"), ("B", "edge")])
def test_tr_equals_dense_bruteforce_random(seed, variant, rule):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 16))
    R = synth.random_r(rng, n, float(rng.uniform(0.15, 0.6)), max_overhang=60,
                       allow_nonpositive=(seed % 3 == 0))
    fuzz = int(rng.integers(0, 40))
    D, iters, _ = bruteforce.tr_dense(R, fuzz, variant, rule)
    S, it2, trace = oracle.transitive_reduce(R, fuzz, variant, rule)
    assert np.array_equal(_s_packed(S), _dense_from_bf(D, n))
    assert it2 == iters
    assert np.all(np.diff(trace) <= 0)


@pytest.mark.parametrize("seed", range(6))
def test_tr_first_pass_marks_equal_bruteforce(seed):
    rng = np.random.default_rng(300 + seed)
    n = 14
    R = synth.random_r(rng, n, 0.4, max_overhang=50)
    _, _, first = bruteforce.tr_dense(R, 15, "A", "row")
    marks = oracle.tr_pass_marks(R, 15)
    got = set()
    for i in range(n):
        for e in range(int(R.rowptr[i]), int(R.rowptr[i + 1])):
            if marks[e]:
                got.add((i, int(R.col[e])))
    assert got == first


@pytest.mark.parametrize("seed", range(10))
def test_tr_closed_dag_reduces_to_networkx_transitive_reduction(seed):
    nx = pytest.importorskip("networkx")
    rng = np.random.default_rng(500 + seed)
    n = 12
    G = nx.DiGraph()
    G.add_nodes_from(range(n))
    for i in range(n):
        for j in range(i + 1, n):
            if rng.random() < 0.25:
                G.add_edge(i, j)
    Cl = nx.transitive_closure_dag(G)
    Tr = nx.transitive_reduction(Cl)
    oh = {e: int(rng.integers(1, 50)) for e in Cl.edges}
    rows = [u for u, v in Cl.edges]
    cols = [v for u, v in Cl.edges]
    vals = [oh[e] << 2 for e in Cl.edges]
    R = synth.coo_to_csr(n, n, rows, cols, vals)
    S, iters, _ = oracle.transitive_reduce(R, 2 * 50)
    got = set()
    for i in range(n):
        for e in range(int(S.rowptr[i]), int(S.rowptr[i + 1])):
            got.add((i, int(S.col[e])))
    assert got == set(Tr.edges)
    assert iters == (2 if got != set(Cl.edges) else 1)


@pytest.mark.parametrize("seed", [21, 22, 23])
def test_tr_error_free_reads_give_the_chain(seed):
    rng = np.random.default_rng(seed)
    g = synth.random_genome(rng, 60_000)
    reads = synth.sample_reads(rng, g, n_reads=120, length_uniform=(2000, 6000), error_rate=0.0)
    R = synth.overlap_graph(reads.start, reads.end, reads.strand, policy="reads")
    S, iters, _ = oracle.transitive_reduce(R, 1000)
    alive = ~synth.contained_reads(reads.start, reads.end)
    idx = np.nonzero(alive)[0]
    idx = idx[np.argsort(reads.start[idx], kind="stable")]
    expect = set()
    for a, b in zip(idx[:-1], idx[1:]):
        if reads.start[b] < reads.end[a]:
            expect.add((int(a), int(b)))
            expect.add((int(b), int(a)))
    got = set()
    for i in range(S.nrows):
        for e in range(int(S.rowptr[i]), int(S.rowptr[i + 1])):
            got.add((i, int(S.col[e])))
    assert got == expect
    assert iters == 2


def test_tr_invariants_on_noisy_tiny_workload():
    w = synth.make_workload("tiny")
    rng = np.random.default_rng(9)
    Rn = synth.perturb_graph(rng, w.R, jitter=40, false_edges=300, flip_codes=0.05)
    for variant in ("A", "B"):
        S, iters, trace = oracle.transitive_reduce(Rn, w.fuzz, variant)
        # S is a subset of R (values unchanged)
        Rp = {(i, int(Rn.col[e])): int(Rn.val[e]) for i in range(Rn.nrows)
              for e in range(int(Rn.rowptr[i]), int(Rn.rowptr[i + 1]))}
        for i in range(S.nrows):
            for e in range(int(S.rowptr[i]), int(S.rowptr[i + 1])):
                assert Rp[(i, int(S.col[e]))] == int(S.val[e])
        # idempotent: reducing S again deletes nothing
        S2, it2, _ = oracle.transitive_reduce(S, w.fuzz, variant)
        assert it2 == 1 and np.array_equal(S2.col, S.col) and np.array_equal(S2.rowptr, S.rowptr)
        assert np.all(np.diff(trace) <= 0)
        if variant == "B":
            assert iters <= 2


def test_tr_contained_entries_dropped():
    R = synth.coo_to_csr(3, 3, [0, 1, 1, 2], [1, 0, 2, 1],
                         synth.encode_r([0, 5, -3, 7], [0, 0, 0, 0], [0, 0, 0, 0]))
    S, iters, trace = oracle.transitive_reduce(R, 10)
    assert trace[0] == 2
    assert {(0, 1), (1, 2)}.isdisjoint({(i, int(S.col[e])) for i in range(3)
                                        for e in range(int(S.rowptr[i]), int(S.rowptr[i + 1]))})


# ---------------------------------------------------------------------------
# Overlap graph from the seeds of C
# ---------------------------------------------------------------------------

def _reads_from(seqs):
    """Reads object holding the given base arrays (truth fields unused)."""
    lens = np.array([s.size for s in seqs], np.int64)
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    z = np.zeros(len(seqs), np.int64)
    return synth.Reads(np.concatenate(seqs).astype(np.uint8), offs, z, z, z.astype(np.int8))


def _canonical_kmers_unique(g, k=17):
    codes = np.zeros(g.size - k + 1, np.int64)
    rcs = np.zeros_like(codes)
    for q in range(k):
        w = g[q:q + codes.size].astype(np.int64)
        codes = (codes << 2) | w
        rcs = rcs | ((3 - w) << (2 * q))
    canon = np.minimum(codes, rcs)
    return np.unique(canon).size == canon.size


@pytest.mark.parametrize("seed", [61, 66])
def test_r_from_seeds_equals_truth_on_error_free_reads(seed):
    """Error-free reads of a genome whose canonical 17-mers are all distinct:
    every seed places its pair exactly, so R from the seeds of C must equal
    the overlap graph from the true coordinates (pairs overlapping by at
    least min_overlap; contained pairs carry value 0), both strands mixed."""
    rng = np.random.default_rng(seed)
    g = synth.random_genome(rng, 80_000)
    assert _canonical_kmers_unique(g)   # (seeds chosen so that no 17-mer recurs)
    reads = synth.sample_reads(rng, g, n_reads=120, length_uniform=(1500, 7000), error_rate=0.0)
    A, _ = synth.kmer_matrix(reads, 17, 2, 1000, strand_bit=True)
    C = oracle.overlap(A, 1)
    lens = np.diff(reads.offsets)
    T = synth.overlap_graph(reads.start, reads.end, reads.strand, min_overlap=100, policy="edges")
    tval = np.where((T.val >> 2) == 0, 0, T.val)
    # one seed, or both seeds at zero drift (exact reads: every shared k-mer
    # gives the same offset), or a density exact reads far exceed (every
    # position of the overlap but the last 16 starts a shared k-mer)
    for drift, density in ((-1, 0), (0, 0), (0, 5000)):
        R = oracle.r_from_seeds(C, lens, 17, 100, drift, density)
        assert R.col.size > 500 and np.count_nonzero(R.val == 0) > 10
        assert np.array_equal(R.rowptr, T.rowptr)
        assert np.array_equal(R.col, T.col)
        assert np.array_equal(R.val, tval)


def test_r_from_seeds_four_overlap_categories():
    """Hand-built pairs of each category of overlap (Sec. IV-E): forward /
    reverse (same strand, read i's alignment starting after / before read
    j's), inner / outer (reverse-complementary), and contained pairs."""
    rng = np.random.default_rng(63)
    g = synth.random_genome(rng, 9000)
    assert _canonical_kmers_unique(g)
    rcv = synth.revcomp
    # (read i, read j, expected value of R_ij): suffix << 2 | code (o_i << 1 | o_j)
    cases = [
        ("forward", g[0:3000], g[1000:5000], (2000 << 2) | 0b00),
        ("reverse", g[1000:5000], g[0:3000], (1000 << 2) | 0b11),
        ("inner", g[0:3000], rcv(g[1000:5000]), (2000 << 2) | 0b01),
        ("outer", g[1000:5000], rcv(g[0:3000]), (1000 << 2) | 0b10),
        ("inner, i reverse complemented", rcv(g[1000:5000]), g[0:3000], (1000 << 2) | 0b01),
        ("contained", g[0:5000], g[1000:3000], 0),
        ("contained, reverse complement", rcv(g[1000:3000]), g[0:5000], 0),
    ]
    for name, si, sj, want in cases:
        A, _ = synth.kmer_matrix(_reads_from([si, sj]), 17, 2, 10, strand_bit=True)
        C = oracle.overlap(A, 1)
        R = oracle.r_from_seeds(C, [si.size, sj.size], 17, 100)
        assert list(R.rowptr) == [0, 1, 2], name
        assert int(R.col[0]) == 1 and int(R.val[0]) == want, (name, int(R.val[0]) >> 2, int(R.val[0]) & 3)


def test_r_from_seeds_keeps_an_overlap_of_exactly_min_overlap():
    rng = np.random.default_rng(63)
    g = synth.random_genome(rng, 9000)
    si, sj = g[0:3000], g[1000:5000]            # overlap of 2000 bases
    A, _ = synth.kmer_matrix(_reads_from([si, sj]), 17, 2, 10, strand_bit=True)
    C = oracle.overlap(A, 1)
    assert oracle.r_from_seeds(C, [3000, 4000], 17, 2000).col.size == 2
    assert oracle.r_from_seeds(C, [3000, 4000], 17, 2001).col.size == 0


def test_r_from_seeds_is_transpose_consistent_on_noisy_reads():
    """With errors the placement is approximate, but C_ji holds C_ij's seeds
    swapped, so every dovetail pair is described the same way from both
    ends: the reverse edge has code (1 - o_j, 1 - o_i) and both edges span
    L_i + suffix_ij = L_j + suffix_ji bases."""
    w = synth.make_workload("tiny", strand_bit=True)
    C = oracle.overlap(w.A, w.min_shared)
    lens = np.diff(w.reads.offsets)
    R = oracle.r_from_seeds(C, lens, w.k, 200, 150, 16)
    assert R.col.size < oracle.r_from_seeds(C, lens, w.k, 200, 150).col.size < \
        oracle.r_from_seeds(C, lens, w.k, 200).col.size
    n = R.nrows
    val = {}
    for i in range(n):
        for e in range(R.rowptr[i], R.rowptr[i + 1]):
            val[(i, int(R.col[e]))] = int(R.val[e])
    dovetails = 0
    for (i, j), v in val.items():
        assert (j, i) in val
        u = val[(j, i)]
        if v == 0 or u == 0:
            assert v == 0 and u == 0
            continue
        dovetails += 1
        assert (u & 3) == ((1 - (v & 1)) << 1 | (1 - ((v >> 1) & 1)))
        assert lens[i] + (v >> 2) == lens[j] + (u >> 2)
    assert dovetails > 1000


def test_r_from_seeds_second_seed_must_agree():
    """max_drift >= 0: the pair is kept only if its second seed exists, has
    the same relative orientation and an offset within max_drift bases of
    the first seed's; max_drift < 0 uses the first seed alone."""
    def c_of(s0, s1):
        seed = np.array([list(s0) + list(s1), list(s0[::-1]) + list(s1[::-1])], np.int32)
        return types.SimpleNamespace(nrows=2, rowptr=np.array([0, 1, 2]), col=np.array([1, 0], np.int32),
                                     count=np.array([2, 2], np.int32), seed=seed)
    L = [5000, 5000]
    base = (1500 << 1, 500 << 1)                       # offset 1000, same strand
    cases = [((3000 << 1, 2000 << 1), 0, True),        # offset 1000: agrees exactly
             ((3000 << 1, 2030 << 1), 30, True),       # offset 970: within 30
             ((3000 << 1, 2031 << 1), 30, False),      # offset 969: beyond 30
             ((2030 << 1, 3000 << 1), 30, False),      # offset -970: far off
             (((3000 << 1) | 1, 2000 << 1), 1000, False),   # other orientation
             ((-1, -1), 1000, False)]                  # no second seed
    for s1, drift, kept in cases:
        C = c_of(base, s1)
        assert oracle.r_from_seeds(C, L, 17, 100, drift).col.size == (2 if kept else 0), (s1, drift)
        assert oracle.r_from_seeds(C, L, 17, 100, -1).col.size == 2


def test_r_from_seeds_density_of_shared_kmers():
    """min_density > 0: kept iff count * 10000 >= min_density * overlap, the
    overlap being the placed one (here 4000 bases)."""
    L = [5000, 5000]
    seed = np.array([[1500 << 1, 500 << 1, 3000 << 1, 2000 << 1], [500 << 1, 1500 << 1, 2000 << 1, 3000 << 1]],
                    np.int32)                                   # offset 1000: overlap 4000
    for count, density, kept in ((20, 50, True), (19, 50, False), (2, 5, True), (1, 5, False), (1, 0, True)):
        C = types.SimpleNamespace(nrows=2, rowptr=np.array([0, 1, 2]), col=np.array([1, 0], np.int32),
                                  count=np.array([count, count], np.int32), seed=seed)
        got = oracle.r_from_seeds(C, L, 17, 100, 0, density).col.size
        assert got == (2 if kept else 0), (count, density)


def test_r_from_seeds_rejects_a_seed_outside_its_read():
    C = types.SimpleNamespace(nrows=2, rowptr=np.array([0, 1, 2]), col=np.array([1, 0], np.int32),
                              count=np.array([1, 1], np.int32),
                              seed=np.array([[10 << 1, 5 << 1, -1, -1], [5 << 1, 10 << 1, -1, -1]], np.int32))
    oracle.r_from_seeds(C, [100, 100], 17, 10)
    with pytest.raises(ValueError):
        oracle.r_from_seeds(C, [100, 20], 17, 10)


# ---------------------------------------------------------------------------
# A from the reads (k-mer counting, reliable k-mers, A): pinned on the read
# strings themselves (Python strings and a Counter, not 2-bit integers)
# ---------------------------------------------------------------------------
def _kmer_matrix_from_strings(seqs, k, lo, hi, strand_bit):
    """A written from the definitions on strings: canonical = the smaller of
    the k-mer and its reverse complement as strings over ACGT (string order
    = the 2-bit code order), frequency over all windows, reliable in
    [lo, hi], columns = reliable canonical strings in the order they are
    first met reading the reads one after the other, value = the first
    position of the k-mer in the read (with its strand: 1 when the read
    holds the reverse complement)."""
    from collections import Counter
    comp = str.maketrans("ACGT", "TGCA")
    freq = Counter()
    met = []                      # canonical strings, each once, as first met
    per_read = []
    for s in seqs:
        first = {}
        for p in range(len(s) - k + 1):
            km = s[p:p + k]
            rc = km.translate(comp)[::-1]
            can = min(km, rc)
            if freq[can] == 0:
                met.append(can)
            freq[can] += 1
            if can not in first:
                first[can] = (p, 1 if rc < km else 0)
        per_read.append(first)
    cols = [c for c in met if lo <= freq[c] <= hi]
    index = {c: q for q, c in enumerate(cols)}
    rows = []
    for first in per_read:
        ent = sorted((index[c], (p << 1 | st) if strand_bit else p) for c, (p, st) in first.items() if c in index)
        rows.append(ent)
    codes = [int("".join("0123"["ACGT".index(ch)] for ch in c), 4) for c in cols]
    return rows, np.array(codes, dtype=np.uint64)


def _rows_of(A):
    return [list(zip(A.col[A.rowptr[i]:A.rowptr[i + 1]].tolist(), A.val[A.rowptr[i]:A.rowptr[i + 1]].tolist()))
            for i in range(A.nrows)]


@pytest.mark.parametrize("seed,k,lo,hi,strand_bit", [
    (0, 5, 2, 6, False), (1, 5, 2, 6, True), (2, 4, 1, 3, True), (3, 7, 2, 40, True), (4, 1, 1, 1000, True),
    (5, 2, 3, 9, False)])
def test_kmer_matrix_equals_strings(seed, k, lo, hi, strand_bit):
    """Error-prone reads of a small genome with repeats, several k (even k
    has palindromic k-mers: strand 0), bounds and value layouts; reads
    shorter than k have empty rows."""
    rng = np.random.default_rng(900 + seed)
    g = synth.random_genome(rng, 1500)
    g[700:760] = g[100:160]                      # a repeat
    reads = synth.sample_reads(rng, g, n_reads=25, length_uniform=(3, 300), error_rate=0.1, min_len=3)
    # and two reads without a window: k - 1 bases, and none
    short = rng.integers(0, 4, size=k - 1, dtype=np.uint8)
    bases = np.concatenate([reads.bases, short])
    offsets = np.concatenate([reads.offsets, [len(bases), len(bases)]]).astype(np.int64)
    seqs = [bruteforce.bases_to_str(bases[offsets[i]:offsets[i + 1]]) for i in range(len(offsets) - 1)]
    A, codes = oracle.kmer_matrix(bases, offsets, k, lo, hi, strand_bit)
    rows, ref_codes = _kmer_matrix_from_strings(seqs, k, lo, hi, strand_bit)
    assert A.ncols == len(ref_codes) and np.array_equal(codes, ref_codes)
    assert _rows_of(A) == rows
    assert A.rowptr[0] == 0 and A.rowptr[-1] == A.nnz


def test_kmer_matrix_palindromes_and_single_bases():
    """k = 2 on "ACGT": AC/GT are each other's reverse complement (canonical
    AC, strand 0 for AC, 1 for GT), CG is its own (strand 0).  k = 1: A and
    T are one canonical base (A), C and G another (C)."""
    bases = np.array([0, 1, 2, 3], np.uint8)      # ACGT
    off = np.array([0, 4], np.int64)
    A, codes = oracle.kmer_matrix(bases, off, 2, 1, 10, True)
    # windows AC (code 1), CG (6, palindrome), GT (11 -> rc AC = 1, strand 1)
    assert codes.tolist() == [1, 6]
    assert _rows_of(A) == [[(0, 0 << 1 | 0), (1, 1 << 1 | 0)]]   # AC first at 0; CG at 1
    A1, codes1 = oracle.kmer_matrix(bases, off, 1, 1, 10, True)
    assert codes1.tolist() == [0, 1]                               # A (from A and T), C (from C and G)
    assert _rows_of(A1) == [[(0, 0 << 1 | 0), (1, 1 << 1 | 0)]]


def test_kmer_matrix_frequency_counts_repeats_inside_a_read():
    """AAAAA with k = 3: three windows of one k-mer -> frequency 3; kept at
    lo = hi = 3, dropped at hi = 2; the value is the first position."""
    bases = np.zeros(5, np.uint8)
    off = np.array([0, 5], np.int64)
    A, codes = oracle.kmer_matrix(bases, off, 3, 3, 3)
    assert codes.tolist() == [0] and _rows_of(A) == [[(0, 0)]]
    A2, codes2 = oracle.kmer_matrix(bases, off, 3, 1, 2)
    assert A2.ncols == 0 and A2.nnz == 0 and A2.rowptr.tolist() == [0, 0]


def test_kmer_matrix_matches_the_generator_on_the_tiny_workload():
    """The generator's A (torch.unique over canonical codes) is the oracle's."""
    w = synth.make_workload("tiny", strand_bit=True)
    A, codes = oracle.kmer_matrix(w.reads.bases, w.reads.offsets, w.k, w.lo, w.hi, True)
    B, bcodes = synth.kmer_matrix(w.reads, w.k, w.lo, w.hi, strand_bit=True)
    assert np.array_equal(A.rowptr, B.rowptr) and np.array_equal(A.col, B.col) and np.array_equal(A.val, B.val)
    assert np.array_equal(codes, bcodes)


@pytest.mark.parametrize("k,lo,hi,bad_base", [(0, 1, 2, False), (32, 1, 2, False), (5, 0, 2, False),
                                              (5, 3, 2, False), (5, 1, 2, True)])
def test_kmer_matrix_rejects_bad_arguments(k, lo, hi, bad_base):
    bases = np.array([0, 1, 2, 3, 4 if bad_base else 0, 1, 2], np.uint8)
    with pytest.raises(ValueError):
        oracle.kmer_matrix(bases, np.array([0, 7], np.int64), k, lo, hi)


# ---------------------------------------------------------------------------
# Seed-and-extend alignment of C's pairs, and R from its ends
# (Sec. IV-D: Apply(C, Alignment()) and Prune(C, AlignmentScoreLessThan(t)))
# ---------------------------------------------------------------------------

def _full_dp_best(a, b, mat, mis, gap):
    """Every cell of the extension table, no pruning: T(i, j) is the best
    score of aligning a[:i] with b[:j] from T(0, 0) = 0.  Returns the largest
    T and the first cell holding it, scanning i + j upward, then i upward."""
    m, n = len(a), len(b)
    T = [[0] * (n + 1) for _ in range(m + 1)]
    for i in range(m + 1):
        for j in range(n + 1):
            if i == 0 and j == 0:
                continue
            cands = []
            if i and j:
                cands.append(T[i - 1][j - 1] + (mat if a[i - 1] == b[j - 1] else mis))
            if i:
                cands.append(T[i - 1][j] + gap)
            if j:
                cands.append(T[i][j - 1] + gap)
            T[i][j] = max(cands)
    best, at = 0, (0, 0)
    for d in range(m + n + 1):
        for i in range(max(0, d - n), min(m, d) + 1):
            if T[i][d - i] > best:
                best, at = T[i][d - i], (i, d - i)
    return best, at


@pytest.mark.parametrize("seed", range(6))
def test_xdrop_with_unbounded_drop_is_the_full_table(seed):
    """With X beyond any score range nothing is pruned: the extension's
    best and its cell are those of the whole table (random and similar
    pairs, several scoring schemes, empty sequences)."""
    rng = np.random.default_rng(900 + seed)
    for t in range(25):
        m, n = int(rng.integers(0, 36)), int(rng.integers(0, 36))
        a = rng.integers(0, 4, size=m, dtype=np.uint8)
        if t % 2:                                    # b: a with substitutions and shifts
            b = a.copy()
            flip = rng.random(m) < 0.2
            b[flip] = (b[flip] + 1) % 4
            b = np.concatenate([b[: m // 3], rng.integers(0, 4, size=int(rng.integers(0, 3)), dtype=np.uint8),
                                b[m // 3 + int(rng.integers(0, 2)):]])[:n] if m else b
        else:
            b = rng.integers(0, 4, size=n, dtype=np.uint8)
        mat, mis, gap = int(rng.integers(1, 4)), -int(rng.integers(1, 4)), -int(rng.integers(1, 5))
        got = oracle.xdrop_extend(a, b, mat, mis, gap, 10 ** 6)
        assert got == _full_dp_best(list(a), list(b), mat, mis, gap), (seed, t, m, len(b))


def test_xdrop_prunes_a_drop_beyond_x_and_keeps_one_of_exactly_x():
    """50 matches, then 10 bases that cannot match (A against C), then 50
    matches: crossing costs 10, so X = 10 reaches the far end (score 90)
    and X = 9 stops after the first run (score 50)."""
    rng = np.random.default_rng(910)
    p1, p2 = rng.integers(0, 4, size=50, dtype=np.uint8), rng.integers(0, 4, size=50, dtype=np.uint8)
    a = np.concatenate([p1, np.zeros(10, np.uint8), p2])
    b = np.concatenate([p1, np.ones(10, np.uint8), p2])
    assert oracle.xdrop_extend(a, b, 1, -1, -1, 10) == (90, (110, 110))
    assert oracle.xdrop_extend(a, b, 1, -1, -1, 9) == (50, (50, 50))
    assert oracle.xdrop_extend(a, b, 1, -1, -1, 10 ** 6) == _full_dp_best(list(a), list(b), 1, -1, -1)


def test_xdrop_ends_at_the_last_match_before_unrelated_tails():
    """Identical 300 bases followed by tails that never match (all A against
    all C): the extension ends where the identical part does."""
    rng = np.random.default_rng(911)
    p = rng.integers(0, 4, size=300, dtype=np.uint8)
    a = np.concatenate([p, np.zeros(500, np.uint8)])
    b = np.concatenate([p, np.ones(400, np.uint8)])
    for X in (1, 5, 50, 200):
        assert oracle.xdrop_extend(a, b, 1, -1, -1, X) == (300, (300, 300))
    assert oracle.xdrop_extend(a, b, 2, -3, -4, 25) == (600, (300, 300))


def test_xdrop_band_limit():
    """An anti-diagonal with more than 256 cells to consider ends the
    extension with the best so far: with nothing pruned on two identical
    3000-base sequences, anti-diagonal 256 would need 257 cells, so the best
    is that of anti-diagonals 0..255, T(127, 127) = 127; with X = 50 the
    band stays narrow and the extension reaches (3000, 3000)."""
    rng = np.random.default_rng(912)
    p = rng.integers(0, 4, size=3000, dtype=np.uint8)
    assert oracle.xdrop_extend(p, p, 1, -1, -1, 10 ** 6) == (127, (127, 127))
    assert oracle.xdrop_extend(p, p, 1, -1, -1, 50) == (3000, (3000, 3000))
    # one sequence of 255 bases: every anti-diagonal has at most 256 cells
    q = p[:255]
    assert oracle.xdrop_extend(q, p, 1, -1, -1, 10 ** 6) == (255, (255, 255))


def test_xdrop_ties_go_to_the_first_cell():
    """Match 2, gaps -1: AC against CA reaches 1 at (1, 2) (a gap, then
    A = A) and at (2, 1) (a gap, then C = C), both on anti-diagonal 3: the
    smaller i is the end.  A best equalled on a later anti-diagonal does
    not move the end; a larger one does."""
    assert _full_dp_best([0, 1], [1, 0], 2, -1, -1) == (1, (1, 2))
    assert oracle.xdrop_extend(np.array([0, 1], np.uint8), np.array([1, 0], np.uint8), 2, -1, -1, 100) == (1, (1, 2))
    assert oracle.xdrop_extend(np.array([1, 0], np.uint8), np.array([0, 1], np.uint8), 2, -1, -1, 100) == (1, (1, 2))
    # equal best on a later anti-diagonal: A,A against A,C,A -> 2 at (1,1), then (2,3): 2 + (-1) + 2 = 3
    assert oracle.xdrop_extend(np.array([0, 0], np.uint8), np.array([0, 1, 0], np.uint8), 2, -1, -1, 100) == (3, (2, 3))
    # A against A,C: 2 at (1,1); (1,2) = 1 is lower; the end stays (1,1)
    assert oracle.xdrop_extend(np.array([0], np.uint8), np.array([0, 1], np.uint8), 2, -1, -1, 100) == (2, (1, 1))
    # match 1, gap -1: A,C,G against A,G: 1 at (1,1), 0 at (2,1) and (1,2), then G = G:
    # (3,2) = 1 on anti-diagonal 5 ties the best of anti-diagonal 2 and does not replace it
    assert oracle.xdrop_extend(np.array([0, 1, 2], np.uint8), np.array([0, 2], np.uint8), 1, -1, -1, 100) == (1, (1, 1))


def test_xdrop_empty_and_one_sided():
    z = np.zeros(0, np.uint8)
    assert oracle.xdrop_extend(z, z) == (0, (0, 0))
    assert oracle.xdrop_extend(np.array([1, 2, 3], np.uint8), z) == (0, (0, 0))
    assert oracle.xdrop_extend(z, np.array([1], np.uint8)) == (0, (0, 0))
    assert oracle.xdrop_extend(np.array([2], np.uint8), np.array([2], np.uint8)) == (1, (1, 1))


def _r_as_dict(R):
    return {(i, int(R.col[e])): int(R.val[e]) for i in range(R.nrows) for e in range(R.rowptr[i], R.rowptr[i + 1])}


@pytest.mark.parametrize("seed", [61, 66])
def test_r_from_alignment_equals_truth_on_error_free_reads(seed):
    """Error-free reads of a genome whose canonical 17-mers are all distinct:
    every seed extends over exactly the true overlap (the reads end where it
    does), so each pair's score is its overlap length and R from the
    alignment ends is the overlap graph from the true coordinates."""
    rng = np.random.default_rng(seed)
    g = synth.random_genome(rng, 80_000)
    assert _canonical_kmers_unique(g)
    reads = synth.sample_reads(rng, g, n_reads=120, length_uniform=(1500, 7000), error_rate=0.0)
    A, _ = synth.kmer_matrix(reads, 17, 2, 1000, strand_bit=True)
    C = oracle.overlap(A, 1)
    T = synth.overlap_graph(reads.start, reads.end, reads.strand, min_overlap=100, policy="edges")
    tval = np.where((T.val >> 2) == 0, 0, T.val)
    R, score = oracle.r_from_alignment(C, reads.bases, reads.offsets, 17, xdrop=50, min_score=100)
    assert R.nnz > 500 and np.count_nonzero(R.val == 0) > 10
    assert np.array_equal(R.rowptr, T.rowptr) and np.array_equal(R.col, T.col) and np.array_equal(R.val, tval)
    rows = np.repeat(np.arange(C.nrows), np.diff(C.rowptr))
    lo = np.maximum(reads.start[rows], reads.start[C.col])
    hi = np.minimum(reads.end[rows], reads.end[C.col])
    off = rows != C.col
    assert np.array_equal(score[off], (hi - lo)[off]) and np.all(score[~off] == 0)


def test_r_from_alignment_four_overlap_categories_with_errors():
    """The hand-built pairs of each category (Sec. IV-E), error-free and
    then with one substitution every 40 bases in read j: the alignment
    still spans the whole overlap, so the suffix and code are exact; the
    score is the overlap length, less two per substitution inside it."""
    rng = np.random.default_rng(63)
    g = synth.random_genome(rng, 9000)
    assert _canonical_kmers_unique(g)
    rcv = synth.revcomp
    cases = [
        ("forward", g[0:3000], g[1000:5000], (2000 << 2) | 0b00, 2000),
        ("reverse", g[1000:5000], g[0:3000], (1000 << 2) | 0b11, 2000),
        ("inner", g[0:3000], rcv(g[1000:5000]), (2000 << 2) | 0b01, 2000),
        ("outer", g[1000:5000], rcv(g[0:3000]), (1000 << 2) | 0b10, 2000),
        ("inner, i reverse complemented", rcv(g[1000:5000]), g[0:3000], (1000 << 2) | 0b01, 2000),
        ("contained", g[0:5000], g[1000:3000], 0, 2000),
        ("contained, reverse complement", rcv(g[1000:3000]), g[0:5000], 0, 2000),
    ]
    for name, si, sj, want, ov in cases:
        for noisy in (False, True):
            sj2 = sj.copy()
            if noisy:          # substitutions away from both ends of j
                pos = np.arange(20, sj2.size - 20, 40)
                sj2[pos] = (sj2[pos] + 1) % 4
            reads = _reads_from([si, sj2])
            A, _ = synth.kmer_matrix(reads, 17, 2, 10, strand_bit=True)
            C = oracle.overlap(A, 1)
            R, score = oracle.r_from_alignment(C, reads.bases, reads.offsets, 17, xdrop=30, min_score=100)
            assert list(R.rowptr) == [0, 1, 2], (name, noisy)
            assert int(R.col[0]) == 1 and int(R.val[0]) == want, (name, noisy, int(R.val[0]) >> 2, int(R.val[0]) & 3)
            assert score[0] == 0 and score[3] == 0          # the diagonal
            if not noisy:
                assert score[1:3].tolist() == [ov, ov], name
            else:
                # the substitutions of j that fall inside the overlap
                assert score[1] == score[2] and ov - 2 * 60 < score[1] < ov - 2 * 40, (name, score)


def test_r_from_alignment_keeps_a_score_of_exactly_min_score():
    rng = np.random.default_rng(63)
    g = synth.random_genome(rng, 9000)
    reads = _reads_from([g[0:3000], g[1000:5000]])
    A, _ = synth.kmer_matrix(reads, 17, 2, 10, strand_bit=True)
    C = oracle.overlap(A, 1)
    assert oracle.r_from_alignment(C, reads.bases, reads.offsets, 17, min_score=2000)[0].nnz == 2
    assert oracle.r_from_alignment(C, reads.bases, reads.offsets, 17, min_score=2001)[0].nnz == 0


def test_r_from_alignment_matches_full_tables_on_short_noisy_pairs():
    """Short pairs (under 256 bases, so no anti-diagonal reaches the band
    limit of 256 cells) with substitutions and deletions, X unbounded: each pair's score
    and R entry follow from the whole extension tables of the two sides of
    its seed, built here from the read strings (read j reverse complemented
    when the strands differ)."""
    rng = np.random.default_rng(64)
    checked = 0
    for t in range(12):
        g = synth.random_genome(rng, 2000)
        s0 = int(rng.integers(0, 400))
        si = g[s0:s0 + int(rng.integers(150, 256))]
        s1 = s0 + int(rng.integers(-100, 120))
        s1 = max(0, s1)
        sj = g[s1:s1 + int(rng.integers(150, 256))].copy()
        flip = rng.random(sj.size) < 0.05
        sj[flip] = (sj[flip] + 1) % 4
        keep = rng.random(sj.size) > 0.03
        sj = sj[keep]
        rc = bool(t % 2)
        if rc:
            sj = synth.revcomp(sj)
        reads = _reads_from([si, sj])
        A, _ = synth.kmer_matrix(reads, 17, 2, 10, strand_bit=True)
        C = oracle.overlap(A, 1)
        R, score = oracle.r_from_alignment(C, reads.bases, reads.offsets, 17, 2, -3, -2, 10 ** 6, min_score=-10 ** 9)
        Rd = _r_as_dict(R)
        for i in range(2):
            for e in range(C.rowptr[i], C.rowptr[i + 1]):
                j = int(C.col[e])
                if j == i:
                    continue
                x, y = reads.read(i), reads.read(j)
                pa, pb = int(C.seed[e][0]), int(C.seed[e][1])
                flipped = (pa & 1) != (pb & 1)
                yo = synth.revcomp(y) if flipped else y
                pi = pa >> 1
                q = (len(y) - 17 - (pb >> 1)) if flipped else (pb >> 1)
                sr, (ear, ebr) = _full_dp_best(list(x[pi + 17:]), list(yo[q + 17:]), 2, -3, -2)
                sl, (eal, ebl) = _full_dp_best(list(x[:pi][::-1]), list(yo[:q][::-1]), 2, -3, -2)
                assert score[e] == sl + 2 * 17 + sr
                bi, bj = pi - eal, q - ebl                       # alignment starts
                ri, rj = len(x) - (pi + 17 + ear), len(y) - (q + 17 + ebr)   # unaligned right ends
                if (bi <= bj and ri <= rj) or (bj <= bi and rj <= ri):
                    want = 0
                elif bi > bj:        # forward (same strand) or inner
                    want = ((rj - ri) << 2) | (1 if flipped else 0)
                else:                # reverse or outer
                    want = ((bj - bi) << 2) | (2 if flipped else 3)
                assert Rd[(i, j)] == want, (t, i, j)
                checked += 1
    assert checked >= 16


def test_r_from_alignment_on_noisy_reads_is_symmetric_and_finds_true_overlaps():
    """15% errors: C_ji holds C_ij's seeds swapped, and the two extensions
    of the swapped pair are the same tables transposed (and complemented
    when the strands differ), so the scores agree both ways.  Scores where
    unrelated bases lose on average (match 1, mismatch -1, gap -2): every
    pair scoring at least 100 is a true overlap."""
    w = synth.make_workload("tiny", strand_bit=True)
    C = oracle.overlap(w.A, w.min_shared)
    R, score = oracle.r_from_alignment(C, w.reads.bases, w.reads.offsets, w.k, 1, -1, -2, 25, min_score=100)
    sc = {}
    for i in range(C.nrows):
        for e in range(C.rowptr[i], C.rowptr[i + 1]):
            sc[(i, int(C.col[e]))] = int(score[e])
    assert all(sc[(j, i)] == s for (i, j), s in sc.items())
    st, en = w.reads.start, w.reads.end
    Rd = _r_as_dict(R)
    assert len(Rd) > 2000
    true = sum(min(en[i], en[j]) - max(st[i], st[j]) > 0 for (i, j) in Rd)
    assert true == len(Rd)
    assert all((j, i) in Rd for (i, j) in Rd)


def test_r_from_alignment_rejects_bad_arguments():
    rng = np.random.default_rng(63)
    g = synth.random_genome(rng, 9000)
    reads = _reads_from([g[0:3000], g[1000:5000]])
    A, _ = synth.kmer_matrix(reads, 17, 2, 10, strand_bit=True)
    C = oracle.overlap(A, 1)
    ok = dict(match=1, mismatch=-1, gap=-2, xdrop=25)
    oracle.r_from_alignment(C, reads.bases, reads.offsets, 17, **ok)
    for bad in (dict(match=0), dict(match=8), dict(mismatch=1), dict(mismatch=-1025), dict(gap=0),
                dict(gap=-1025), dict(xdrop=-1), dict(xdrop=(1 << 20) + 1)):
        with pytest.raises(ValueError):
            oracle.r_from_alignment(C, reads.bases, reads.offsets, 17, **{**ok, **bad})
    b = reads.bases.copy()
    b[7] = 4                                           # a base outside 0..3
    with pytest.raises(ValueError):
        oracle.r_from_alignment(C, b, reads.offsets, 17, **ok)
    with pytest.raises(ValueError):                    # offsets that do not end at the bases' end
        oracle.r_from_alignment(C, reads.bases[:-1], reads.offsets, 17, **ok)
    C2 = types.SimpleNamespace(**vars(C))
    C2.seed = C.seed.copy()
    C2.seed[1, 1] = (3990 << 1)                        # a seed past the end of read 1 (4000 bases)
    with pytest.raises(ValueError):
        oracle.r_from_alignment(C2, reads.bases, reads.offsets, 17, **ok)
