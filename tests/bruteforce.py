"""Brute-force references used to pin the oracle on tiny inputs.

They are written from the definitions directly and in a different form from
the oracle:

* overlap_from_reads works on the read strings themselves (not on A): it
  lists the reliable canonical k-mers of every read as strings and
  intersects the sets of every pair of reads.  So it checks both the oracle
  and the generator's A.
* tr_dense runs the reduction on dense n x n tables with a full triple loop.
"""
from __future__ import annotations

from collections import Counter

import numpy as np

_COMP = str.maketrans("ACGT", "TGCA")


def bases_to_str(b) -> str:
    return "".join("ACGT"[int(x)] for x in b)


def canonical(kmer: str) -> str:
    rc = kmer.translate(_COMP)[::-1]
    return min(kmer, rc)


def overlap_from_reads(reads, k: int, lo: int, hi: int, min_shared: int):
    """Dict {(i, j): (count, (p_i0, p_j0, p_i1, p_j1))} for every read pair
    (diagonal included) sharing >= min_shared reliable k-mers.  The kept
    position pairs belong to the two shared canonical k-mers met first when
    the reads are read one after the other (A's column order); a position
    is the first start of that k-mer in the read as sequenced."""
    seqs = [bases_to_str(reads.read(i)) for i in range(reads.n)]
    freq = Counter()
    met = {}                      # canonical k-mer -> when it was first met
    per_read = []
    for s in seqs:
        first = {}
        for p in range(len(s) - k + 1):
            c = canonical(s[p:p + k])
            freq[c] += 1
            met.setdefault(c, len(met))
            if c not in first:
                first[c] = p
        per_read.append(first)
    reliable = {c for c, f in freq.items() if lo <= f <= hi}
    sets = [{c: p for c, p in fr.items() if c in reliable} for fr in per_read]
    keys = [set(s) for s in sets]
    out = {}
    n = len(seqs)
    for i in range(n):
        for j in range(n):
            shared = keys[i] & keys[j]
            if len(shared) < min_shared or not shared:
                continue
            srt = sorted(shared, key=met.__getitem__)
            s0 = srt[0]
            seed = [sets[i][s0], sets[j][s0], -1, -1]
            if len(srt) > 1:
                s1 = srt[1]
                seed[2], seed[3] = sets[i][s1], sets[j][s1]
            out[(i, j)] = (len(shared), tuple(seed))
    return out, len(reliable)


def csr_to_dense_vals(M, absent=None):
    n = M.nrows
    D = [[absent] * M.ncols for _ in range(n)]
    for i in range(n):
        for e in range(int(M.rowptr[i]), int(M.rowptr[i + 1])):
            D[i][int(M.col[e])] = int(M.val[e])
    return D


def tr_dense(R, fuzz: int, variant: str = "A", rule: str = "row"):
    """Transitive reduction on a dense table of packed R values.

    Returns (dense table of survivors, iterations, marks of the first pass).
    Value packing: (overhang << 2) | (o_src << 1) | o_dst.
    """
    n = R.nrows
    D = csr_to_dense_vals(R)
    for i in range(n):
        for j in range(n):
            if D[i][j] is not None and (D[i][j] >> 2) <= 0:
                D[i][j] = None
    iters = 0
    first_marks = None
    while True:
        iters += 1
        rowmax = [max([D[i][j] >> 2 for j in range(n) if D[i][j] is not None], default=0)
                  for i in range(n)]
        marks = []
        for i in range(n):
            for j in range(n):
                rij = D[i][j]
                if rij is None:
                    continue
                best = None
                for kk in range(n):
                    rik, rkj = D[i][kk], D[kk][j]
                    if rik is None or rkj is None:
                        continue
                    if (rik & 1) != ((rkj >> 1) & 1):          # heads at kk must be opposite
                        continue
                    s = (rik >> 2) + (rkj >> 2)
                    code = (((rik >> 1) & 1) << 1) | (rkj & 1)
                    if variant == "B" and code != (rij & 3):
                        continue
                    cand = (s, code)
                    if best is None or cand < best:
                        best = cand
                lim = ((rij >> 2) if rule == "edge" else rowmax[i]) + fuzz
                if best is not None and best[1] == (rij & 3) and best[0] <= lim:
                    marks.append((i, j))
        if first_marks is None:
            first_marks = set(marks)
        for (i, j) in marks:
            D[i][j] = None
        if not marks:
            return D, iters, first_marks
