"""Seeded synthetic long-read workloads: genomes, reads, the k-mer matrix A and
the overlap graph R.

This module is the input generator shared by the CPU oracle and the HIP path.
It holds none of the method's arithmetic (no A*A^T, no transitive reduction):
it only simulates sequencing and builds the two input matrices the paper's
pipeline hands to its sparse products.

* Reads, reverse complements and canonical k-mers follow Sec. II (canonical
  form = the lexicographically smaller of a k-mer and its reverse complement).
* A (reads x reliable k-mers, value = position of the k-mer in the read)
  follows Sec. IV-C/IV-D: k-mers seen once, or more often than a bound, are
  not reliable and get no column.
* R stands in for the aligned-and-pruned overlap matrix of Sec. IV-D/IV-E.
  Overhang ("overlap suffix") and orientation come from the true read
  coordinates, which is what a perfect aligner would report.

Encodings (shared by every consumer):
  bases       uint8 0..3 for A,C,G,T; a k-mer packs its first base in the most
              significant 2 bits, so integer order equals lexicographic order.
  A           CSR: rowptr int64[n+1], col int32 (sorted, unique per row),
              val int32 (0-based start of the k-mer in the read as sequenced;
              the smallest such start if the k-mer recurs in the read).
  R           CSR n x n: val int32 = (overhang << 2) | (o_src << 1) | o_dst,
              row = source read.  o = 0: the read is traversed as sequenced,
              o = 1: as its reverse complement.  A contained pair is stored
              with overhang 0 (contained overlaps are discarded by the
              reduction itself).

All randomness comes from numpy.random.default_rng(seed); the heavy but
deterministic transforms (k-mer extraction, counting, sorting) run in torch on
the requested device and give identical results on CPU and GPU.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

K_DEFAULT = 17


# ----------------------------------------------------------------------------
# Genomes
# ----------------------------------------------------------------------------

def random_genome(rng: np.random.Generator, length: int) -> np.ndarray:
    """iid uniform A/C/G/T genome (uint8 codes)."""
    return rng.integers(0, 4, size=int(length), dtype=np.uint8)


def revcomp(seq: np.ndarray) -> np.ndarray:
    """Reverse complement of a uint8 base array (A<->T, C<->G)."""
    return (3 - seq[::-1]).astype(np.uint8)


def _mutate(rng: np.random.Generator, seq: np.ndarray, rate: float) -> np.ndarray:
    out = seq.copy()
    hit = rng.random(out.size) < rate
    out[hit] = (out[hit] + rng.integers(1, 4, size=int(hit.sum()))) % 4
    return out.astype(np.uint8)


def _place_nonoverlapping(rng: np.random.Generator, genome_len: int,
                          seg_lens: np.ndarray) -> np.ndarray:
    """Uniform non-overlapping start positions for segments (in given order)."""
    total = int(seg_lens.sum())
    free = genome_len - total
    if free < 0:
        raise ValueError("repeat copies do not fit in the genome")
    gaps = np.sort(rng.integers(0, free + 1, size=seg_lens.size))
    return gaps + np.concatenate([[0], np.cumsum(seg_lens)[:-1]])


def insert_repeats(rng: np.random.Generator, genome: np.ndarray,
                   families: Sequence[tuple]) -> np.ndarray:
    """Write repeat copies over non-overlapping uniform positions.

    families: (unit_length, copies, divergence) per family.  Each copy is the
    family unit with iid substitutions at rate `divergence`; half the copies
    are written reverse-complemented.  The genome length does not change.
    """
    g = genome.copy()
    units, lens = [], []
    for unit_len, copies, div in families:
        unit = random_genome(rng, unit_len)
        for _ in range(int(copies)):
            c = _mutate(rng, unit, div)
            if rng.random() < 0.5:
                c = revcomp(c)
            units.append(c)
            lens.append(unit_len)
    if not units:
        return g
    order = rng.permutation(len(units))
    seg_lens = np.asarray(lens, dtype=np.int64)[order]
    starts = _place_nonoverlapping(rng, g.size, seg_lens)
    for s, idx in zip(starts, order):
        u = units[idx]
        g[s:s + u.size] = u
    return g


# ----------------------------------------------------------------------------
# Reads
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Reads:
    """Concatenated read bases plus the ground truth of every read."""
    bases: np.ndarray      # uint8, all reads back to back
    offsets: np.ndarray    # int64[n+1]
    start: np.ndarray      # int64[n]  genome start of the fragment
    end: np.ndarray        # int64[n]  genome end (exclusive)
    strand: np.ndarray     # int8[n]   0 forward, 1 reverse complement

    @property
    def n(self) -> int:
        return int(self.start.size)

    def read(self, i: int) -> np.ndarray:
        return self.bases[self.offsets[i]:self.offsets[i + 1]]


def sample_reads(rng: np.random.Generator, genome: np.ndarray, *,
                 n_reads: Optional[int] = None, coverage: Optional[float] = None,
                 length_uniform: Optional[tuple] = None,
                 length_lognormal_mean: Optional[float] = None,
                 sigma: float = 0.5, error_rate: float = 0.15,
                 rc_fraction: float = 0.5, min_len: int = 500) -> Reads:
    """Sample error-prone long reads from a genome.

    Lengths are uniform integers in `length_uniform` or lognormal with the
    given mean (mu = ln(mean) - sigma^2/2), clipped to [min_len, G].  Starts
    are uniform, so every fragment lies inside the genome.  A fraction
    `rc_fraction` of reads are reverse-complemented.  Each fragment base
    independently, with probability `error_rate`, is substituted, preceded
    by an inserted random base, or deleted (equally likely).
    """
    G = int(genome.size)

    def draw_lengths(cnt):
        if length_uniform is not None:
            lo, hi = length_uniform
            L = rng.integers(lo, hi + 1, size=cnt)
        else:
            mu = math.log(length_lognormal_mean) - sigma * sigma / 2.0
            L = np.rint(rng.lognormal(mu, sigma, size=cnt)).astype(np.int64)
        return np.clip(L, min(min_len, G), G).astype(np.int64)

    if n_reads is not None:
        lens = draw_lengths(n_reads)
    else:
        target = coverage * G
        chunks, tot = [], 0
        mean_len = (np.mean(length_uniform) if length_uniform is not None
                    else length_lognormal_mean)
        while tot < target:
            need = max(16, int((target - tot) / mean_len * 1.1) + 1)
            L = draw_lengths(need)
            cs = np.cumsum(L) + tot
            cut = int(np.searchsorted(cs, target, side="left")) + 1
            L = L[:cut]
            chunks.append(L)
            tot += int(L.sum())
        lens = np.concatenate(chunks)
    n = int(lens.size)
    starts = (rng.random(n) * (G - lens + 1)).astype(np.int64)
    strand = (rng.random(n) < rc_fraction).astype(np.int8)

    # Gather fragments (reverse complement where strand == 1).
    frag_off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    T = int(frag_off[-1])
    rid = np.repeat(np.arange(n, dtype=np.int64), lens)
    within = np.arange(T, dtype=np.int64) - frag_off[rid]
    rcmask = strand[rid].astype(bool)
    gpos = np.where(rcmask, starts[rid] + lens[rid] - 1 - within, starts[rid] + within)
    frag = genome[gpos]
    frag = np.where(rcmask, 3 - frag, frag).astype(np.uint8)
    del within, gpos, rcmask

    # Sequencing errors.
    u = rng.random(T)
    err = u < error_rate
    typ = rng.integers(0, 3, size=T, dtype=np.int8)
    sub = err & (typ == 0)
    ins = err & (typ == 1)
    dele = err & (typ == 2)
    del u, typ, err
    frag[sub] = (frag[sub] + rng.integers(1, 4, size=int(sub.sum()), dtype=np.uint8)) % 4
    reps = (1 + ins.astype(np.int8) - dele.astype(np.int8)).astype(np.int64)
    out = np.repeat(frag, reps)
    first = np.cumsum(reps) - reps
    ins_at = first[ins]
    out[ins_at] = rng.integers(0, 4, size=ins_at.size, dtype=np.uint8)
    new_lens = np.bincount(rid, weights=reps, minlength=n).astype(np.int64)
    offsets = np.concatenate([[0], np.cumsum(new_lens)]).astype(np.int64)
    return Reads(bases=out.astype(np.uint8), offsets=offsets, start=starts,
                 end=starts + lens, strand=strand)


# ----------------------------------------------------------------------------
# A: reads x reliable k-mers (GenerateA)
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class CSR:
    nrows: int
    ncols: int
    rowptr: np.ndarray   # int64[nrows+1]
    col: np.ndarray      # int32[nnz]
    val: np.ndarray      # int32[nnz]

    @property
    def nnz(self) -> int:
        return int(self.col.size)

    def row(self, i):
        a, b = int(self.rowptr[i]), int(self.rowptr[i + 1])
        return self.col[a:b], self.val[a:b]


def kmer_matrix(reads: Reads, k: int = K_DEFAULT, lo: int = 2, hi: int = 8,
                device: str = "cpu", strand_bit: bool = False) -> tuple:
    """Build A from reads.  Returns (A, kmer_codes) where kmer_codes[c] is the
    canonical 2-bit code of column c.

    Frequency = occurrences of the canonical k-mer over all reads (repeats
    inside a read count); a k-mer is reliable if lo <= frequency <= hi.
    Column order = first occurrence among reliable k-mers: by the first read
    holding the k-mer, then by its smallest position there.
    strand_bit: A's value is (position << 1) | strand instead of the
    position, strand = 1 where the read holds the reverse complement of the
    canonical k-mer (the orientation the overlap graph is derived from).
    """
    import torch
    dev = torch.device(device)
    n = reads.n
    offs = torch.from_numpy(reads.offsets).to(dev)
    b = torch.from_numpy(reads.bases).to(dev).to(torch.int64)
    T = int(b.numel())
    lens = offs[1:] - offs[:-1]
    if T < k:
        empty = CSR(n, 0, np.zeros(n + 1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32))
        return empty, np.zeros(0, np.int64)
    W = T - k + 1
    fwd = torch.zeros(W, dtype=torch.int64, device=dev)
    rc = torch.zeros(W, dtype=torch.int64, device=dev)
    for q in range(k):
        w = b[q:q + W]
        fwd = (fwd << 2) | w
        rc = rc | ((3 - w) << (2 * q))
    canon = torch.minimum(fwd, rc)
    strand = (rc < fwd) if strand_bit else None
    del fwd, rc
    rid = torch.repeat_interleave(torch.arange(n, device=dev), lens)[:W]
    pos = torch.arange(W, device=dev) - offs[rid]
    valid = pos + k <= lens[rid]
    canon, rid, pos = canon[valid], rid[valid], pos[valid]
    if strand is not None:
        pos = (pos << 1) | strand[valid].to(torch.int64)
    uniq, inv, cnt = torch.unique(canon, sorted=True, return_inverse=True, return_counts=True)
    reliable = (cnt >= lo) & (cnt <= hi)
    # the kept windows are in (read, position) order: a k-mer's first
    # occurrence is its smallest window index
    first = torch.full((uniq.numel(),), canon.numel(), dtype=torch.int64, device=dev)
    first.scatter_reduce_(0, inv, torch.arange(canon.numel(), device=dev), reduce="amin")
    rel_idx = torch.nonzero(reliable).flatten()
    by_first = rel_idx[torch.argsort(first[rel_idx])]
    m = int(by_first.numel())
    colmap = torch.full((uniq.numel(),), -1, dtype=torch.int64, device=dev)
    colmap[by_first] = torch.arange(m, device=dev)
    keep = reliable[inv]
    col = colmap[inv][keep]
    rid, pos = rid[keep], pos[keep]
    key = rid * max(m, 1) + col
    skey, order = torch.sort(key, stable=True)
    first = torch.ones_like(skey, dtype=torch.bool)
    if skey.numel() > 1:
        first[1:] = skey[1:] != skey[:-1]
    sel = order[first]
    r_rid, r_col, r_pos = rid[sel], col[sel], pos[sel]
    rowcnt = torch.bincount(r_rid, minlength=n)
    rowptr = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    rowptr[1:] = torch.cumsum(rowcnt, 0)
    A = CSR(n, m, rowptr.cpu().numpy(), r_col.to(torch.int32).cpu().numpy(),
            r_pos.to(torch.int32).cpu().numpy())
    return A, uniq[by_first].cpu().numpy()


# ----------------------------------------------------------------------------
# R: overlap graph from the true coordinates
# ----------------------------------------------------------------------------

def encode_r(oh, o_src, o_dst):
    """Pack overhang and the two end orientations into R's int32 value."""
    oh = np.asarray(oh, dtype=np.int64)
    return ((oh << 2) | (np.asarray(o_src, np.int64) << 1) | np.asarray(o_dst, np.int64)).astype(np.int32)


def decode_r(val):
    v = np.asarray(val, dtype=np.int64)
    return v >> 2, (v >> 1) & 1, v & 1


def contained_reads(start: np.ndarray, end: np.ndarray) -> np.ndarray:
    """Boolean mask of reads whose interval lies inside another read's.
    Identical intervals: the higher index counts as contained."""
    n = start.size
    order = np.lexsort((np.arange(n), -end, start))   # by start, then longer first, then index
    e_sorted = end[order]
    run_max = np.maximum.accumulate(np.concatenate([[-1], e_sorted[:-1]]))
    cont_sorted = e_sorted <= run_max
    out = np.zeros(n, dtype=bool)
    out[order] = cont_sorted
    return out


def overlap_graph(start: np.ndarray, end: np.ndarray, strand: np.ndarray, *,
                  min_overlap: int = 1, policy: str = "edges") -> CSR:
    """Overlap matrix R from true read intervals [start, end) and strands.

    For a dovetail pair with read a left of read b (s_a < s_b, e_a < e_b):
      R[a, b] = (overhang e_b - e_a, code (strand_a, strand_b))
      R[b, a] = (overhang s_b - s_a, code (1 - strand_b, 1 - strand_a))
    i.e. walking the genome left to right visits a then b with the reads in
    their sequencing orientation, and walking it right to left visits b then
    a reverse-complemented.  Contained pairs: policy "edges" keeps them with
    overhang 0 in both directions (the reduction discards them); policy
    "reads" removes every read that lies inside another one.
    Only pairs whose true overlap is >= min_overlap bp are kept.
    """
    start = np.asarray(start, np.int64)
    end = np.asarray(end, np.int64)
    strand = np.asarray(strand, np.int64)
    n = start.size
    alive = np.ones(n, dtype=bool)
    if policy == "reads":
        alive = ~contained_reads(start, end)
    elif policy != "edges":
        raise ValueError(policy)
    order = np.lexsort((np.arange(n), -end, start))
    order = order[alive[order]]
    s_o, e_o = start[order], end[order]
    # partners of sorted read a: later reads b whose start is < e_a - min_overlap + 1
    hi = np.searchsorted(s_o, e_o - min_overlap, side="right")
    cnt = np.maximum(hi - (np.arange(order.size) + 1), 0)
    a_idx = np.repeat(np.arange(order.size), cnt)
    b_idx = (np.arange(a_idx.size) - np.repeat(np.cumsum(cnt) - cnt, cnt)) + a_idx + 1
    a, b = order[a_idx], order[b_idx]
    ov = np.minimum(end[a], end[b]) - np.maximum(start[a], start[b])
    ok = ov >= min_overlap
    a, b = a[ok], b[ok]
    contained = end[b] <= end[a]       # b inside a (a sorts first: s_a <= s_b, ties longer first)
    oh_ab = np.where(contained, 0, end[b] - end[a])
    oh_ba = np.where(contained, 0, start[b] - start[a])
    oh_ba = np.where(~contained & (oh_ba <= 0), 0, oh_ba)
    rows = np.concatenate([a, b])
    cols = np.concatenate([b, a])
    vals = np.concatenate([encode_r(oh_ab, strand[a], strand[b]),
                           encode_r(oh_ba, 1 - strand[b], 1 - strand[a])])
    return coo_to_csr(n, n, rows, cols, vals)


def restrict_to_pattern(R: CSR, rowptr, col, device: str = "cpu") -> CSR:
    """The entries of R whose (row, column) also appears in the pattern
    (rowptr, col) of another n x n matrix, off the diagonal: the overlap
    graph of the true coordinates restricted to the candidate pairs, i.e.
    what a perfect aligner keeps of the candidates (a set intersection of
    two given patterns; nothing of the products is computed here)."""
    import torch
    dev = torch.device(device)
    n = R.nrows
    rp = torch.as_tensor(np.asarray(R.rowptr), device=dev)
    rr = torch.repeat_interleave(torch.arange(n, device=dev), rp[1:] - rp[:-1])
    rkey = rr * n + torch.as_tensor(np.asarray(R.col), device=dev).to(torch.int64)
    crp = torch.as_tensor(rowptr, device=dev).to(torch.int64)
    cr = torch.repeat_interleave(torch.arange(n, device=dev), crp[1:] - crp[:-1])
    cc = torch.as_tensor(col, device=dev).to(torch.int64)
    off = cr != cc
    ckey = cr[off] * n + cc[off]
    keep = torch.isin(rkey, ckey)
    rows = rr[keep]
    out_rp = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    out_rp[1:] = torch.cumsum(torch.bincount(rows, minlength=n), 0)
    kp = keep.cpu().numpy()
    return CSR(n, n, out_rp.cpu().numpy(), np.asarray(R.col)[kp], np.asarray(R.val)[kp])


def coo_to_csr(nrows: int, ncols: int, rows, cols, vals) -> CSR:
    rows = np.asarray(rows, np.int64)
    cols = np.asarray(cols, np.int64)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], np.asarray(vals)[order]
    rowptr = np.zeros(nrows + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=nrows), out=rowptr[1:])
    return CSR(nrows, ncols, rowptr, cols.astype(np.int32), vals.astype(np.int32))


def perturb_graph(rng: np.random.Generator, R: CSR, *, jitter: int = 0,
                  false_edges: int = 0, max_overhang: int = 10000,
                  flip_codes: float = 0.0) -> CSR:
    """Noisy R: +-jitter bp on overhangs (kept >= 1 where it was >= 1),
    random false edges added in transpose-consistent pairs
    ((i,j) with code (x,y) and (j,i) with code (1-y,1-x)), and a fraction of
    entries with a random code."""
    n = R.nrows
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(R.rowptr))
    cols = R.col.astype(np.int64)
    oh, os_, od = decode_r(R.val)
    if jitter:
        j = rng.integers(-jitter, jitter + 1, size=oh.size)
        oh = np.where(oh >= 1, np.maximum(oh + j, 1), oh)
    if flip_codes > 0:
        f = rng.random(oh.size) < flip_codes
        os_ = np.where(f, rng.integers(0, 2, oh.size), os_)
        od = np.where(f, rng.integers(0, 2, oh.size), od)
    vals = encode_r(oh, os_, od)
    if false_edges and n >= 2:
        fi = rng.integers(0, n, size=false_edges)
        fj = rng.integers(0, n - 1, size=false_edges)
        fj = np.where(fj >= fi, fj + 1, fj)
        x = rng.integers(0, 2, false_edges)
        y = rng.integers(0, 2, false_edges)
        o1 = rng.integers(1, max_overhang, false_edges)
        o2 = rng.integers(1, max_overhang, false_edges)
        rows = np.concatenate([rows, fi, fj])
        cols = np.concatenate([cols, fj, fi])
        vals = np.concatenate([vals, encode_r(o1, x, y), encode_r(o2, 1 - y, 1 - x)])
    # drop duplicate (row, col) keeping the first occurrence
    key = rows * n + cols
    _, first = np.unique(key, return_index=True)
    return coo_to_csr(n, n, rows[first], cols[first], vals[first])


# ----------------------------------------------------------------------------
# Random sparse inputs for edge-case tests
# ----------------------------------------------------------------------------

def random_a(rng: np.random.Generator, n: int, m: int, density: float,
             max_pos: int = 100000, dense_rows: Sequence[int] = (),
             dense_cols: Sequence[int] = ()) -> CSR:
    """Random A with sorted unique columns per row and non-negative values.
    `dense_rows` get every column; `dense_cols` appear in every row."""
    mask = rng.random((n, m)) < density
    for r in dense_rows:
        mask[r, :] = True
    for c in dense_cols:
        mask[:, c] = True
    rows, cols = np.nonzero(mask)
    vals = rng.integers(0, max_pos, size=rows.size)
    return coo_to_csr(n, m, rows, cols, vals)


def random_r(rng: np.random.Generator, n: int, density: float, max_overhang: int = 100,
             allow_nonpositive: bool = False) -> CSR:
    """Random bidirected R (no diagonal) with random overhangs and codes."""
    mask = rng.random((n, n)) < density
    np.fill_diagonal(mask, False)
    rows, cols = np.nonzero(mask)
    lo = -5 if allow_nonpositive else 1
    oh = rng.integers(lo, max_overhang + 1, size=rows.size)
    vals = encode_r(oh, rng.integers(0, 2, rows.size), rng.integers(0, 2, rows.size))
    return coo_to_csr(n, n, rows, cols, vals)


# ----------------------------------------------------------------------------
# Workload recipes shaped like the paper's long-read data
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    reads: Reads
    A: CSR
    R: CSR
    min_shared: int
    fuzz: int
    k: int
    lo: int
    hi: int
    genome_len: int
    error_rate: float = 0.0


def _families_to_cover(rng, genome_len, fraction, unit_range, div_range, copies_range):
    fams, covered = [], 0
    while covered < fraction * genome_len:
        U = int(rng.integers(unit_range[0], unit_range[1] + 1))
        c = int(rng.integers(copies_range[0], copies_range[1] + 1))
        d = float(rng.uniform(*div_range))
        fams.append((U, c, d))
        covered += U * c
    return fams


def make_workload(name: str, seed: Optional[int] = None, device: str = "cpu",
                  policy: str = "edges", scale: float = 1.0, strand_bit: bool = False, **over) -> Workload:
    """Build one of the named workloads.

    tiny   100 kbp iid genome, 200 reads U{2..8} kbp, 15% error, k=17,
           reliable [2,8], min_shared 1, R from all true overlaps >= 1 bp,
           fuzz 1000.
    mid    10 Mbp genome with 300 copies of a 2 kbp repeat at 1% divergence,
           30x, lognormal(mean 10 kbp, sigma 0.5), 15% error, reliable [2,30],
           min_shared 2, R from true overlaps >= 1 kbp, fuzz 1000.
    large  50 Mbp genome with 5% repeats (families of 1-6 kbp units,
           0.5-3% divergence, 10-30 copies), 40x, lognormal(mean 12 kbp),
           12% error, reliable [2,40], min_shared 2, R as for mid.
    batchset  one set of the 64-set batch: genome log-uniform in
           [50 kbp, 5 Mbp], 10-50x, lognormal(mean 8 kbp), 15% error, else as
           tiny (reliable [2,8], min_shared 1, R from overlaps >= 1 bp).
    `scale` multiplies the genome length (coverage and read lengths kept).
    `strand_bit`: A's values carry the k-mer strand (see kmer_matrix).
    """
    base_seed = {"tiny": 1000, "mid": 2000, "large": 3000, "batchset": 4000}[name]
    rng = np.random.default_rng(base_seed if seed is None else seed)
    if name == "tiny":
        p = dict(G=100_000, n_reads=200, length_uniform=(2000, 8000), err=0.15,
                 lo=2, hi=8, min_shared=1, min_overlap=1, fuzz=1000, fams=[])
    elif name == "mid":
        p = dict(G=10_000_000, coverage=30, mean_len=10_000, err=0.15, lo=2, hi=30,
                 min_shared=2, min_overlap=1000, fuzz=1000, fams=[(2000, 300, 0.01)])
    elif name == "large":
        p = dict(G=50_000_000, coverage=40, mean_len=12_000, err=0.12, lo=2, hi=40,
                 min_shared=2, min_overlap=1000, fuzz=1000, fams=None)
    else:
        G = int(round(math.exp(rng.uniform(math.log(50_000), math.log(5_000_000)))))
        p = dict(G=G, coverage=float(rng.uniform(10, 50)), mean_len=8000, err=0.15,
                 lo=2, hi=8, min_shared=1, min_overlap=1, fuzz=1000, fams=[])
    p.update(over)
    G = max(int(p["G"] * scale), 20_000)
    if p["fams"] is None:
        fams = _families_to_cover(rng, G, 0.05, (1000, 6000), (0.005, 0.03), (10, 30))
    else:
        fams = [(u, max(1, int(round(c * scale))) if scale != 1.0 else c, d)
                for (u, c, d) in p["fams"]]
    g = insert_repeats(rng, random_genome(rng, G), fams)
    if "n_reads" in p:
        reads = sample_reads(rng, g, n_reads=p["n_reads"], length_uniform=p["length_uniform"],
                             error_rate=p["err"])
    else:
        reads = sample_reads(rng, g, coverage=p["coverage"],
                             length_lognormal_mean=p["mean_len"], error_rate=p["err"])
    A, _ = kmer_matrix(reads, K_DEFAULT, p["lo"], p["hi"], device=device, strand_bit=strand_bit)
    R = overlap_graph(reads.start, reads.end, reads.strand,
                      min_overlap=p["min_overlap"], policy=policy)
    return Workload(name, reads, A, R, p["min_shared"], p["fuzz"], K_DEFAULT,
                    p["lo"], p["hi"], G, p["err"])


def batch_workloads(count: int = 64, seed: int = 4000, device: str = "cpu",
                    scale: float = 1.0) -> list:
    """The uneven sets of the batching workload (one seed per set)."""
    return [make_workload("batchset", seed=seed + s, device=device, scale=scale)
            for s in range(count)]


# ----------------------------------------------------------------------------
# Work counts (units of throughput; computed from the inputs only)
# ----------------------------------------------------------------------------

def overlap_products(A: CSR) -> int:
    """Semiring multiplications in A*A^T: sum over k-mers of (column count)^2."""
    a = np.bincount(A.col, minlength=A.ncols).astype(np.int64)
    return int((a * a).sum())
