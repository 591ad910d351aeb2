"""ctypes front end of the plain C oracle (dibella_oracle.c).

Test infrastructure: only the tests, the smoke check and the benchmark's
CPU-baseline leg import this package.  It shares nothing with the HIP
library.  Inputs are anything with nrows/ncols/rowptr/col/val attributes
(numpy arrays); outputs are plain numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from types import SimpleNamespace

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dibella_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
# A separately built oracle library to load instead: set only by an explicit
# use_library() call (the test that plants mistakes in copies of the oracle
# source calls it in its own child processes, never through the environment).
_LIB_OVERRIDE = None

VARIANT_B = 0x1
RULE_EDGE = 0x2

_lib = None


def use_library(path: str) -> None:
    """Load the oracle from another build of its source (for the child
    processes of the planted-mistake test).  Must be called before any use."""
    global _LIB_OVERRIDE, _lib
    if _lib is not None:
        raise RuntimeError("the oracle library is already loaded")
    _LIB_OVERRIDE = path


def build(force: bool = True) -> str:
    """Compile the oracle with plain gcc -O2 (single thread)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            lib = ctypes.CDLL(_LIB_OVERRIDE)
        else:
            if not os.path.exists(_LIB_PATH):
                build()
            lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i64, i32, u32 = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32
        lib.oracle_overlap_rows.argtypes = [i64, i64, P, P, P, i32, P, i64, P,
                                            P, P, P, P]
        lib.oracle_transpose.argtypes = [i64, i64, P, P, P, P, P, P]
        lib.oracle_overlap_rows_t.argtypes = [i64, i64, P, P, P, P, P, P, i32, P, i64, P,
                                              P, P, P, P]
        lib.oracle_transitive_reduce.argtypes = [i64, P, P, P, i32, u32, P, P, P, P, P, P, i32, P]
        lib.oracle_tr_pass_marks.argtypes = [i64, P, P, P, i32, u32, P, i64, P]
        lib.oracle_r_from_seeds.argtypes = [i64, P, P, P, P, P, i32, i32, i32, i32, P, P, P, P]
        lib.oracle_kmer_matrix.argtypes = [i64, P, P, i32, i32, i32, i32, P, P, P, P, P, P]
        lib.oracle_r_from_alignment.argtypes = [i64, P, P, P, P, P, i32, i32, i32, i32, i32, i32, P, P, P, P, P]
        lib.oracle_xdrop_extend.argtypes = [P, i64, P, i64, i32, i32, i32, i32, P, P]
        lib.oracle_xdrop_extend.restype = i64
        lib.oracle_free.argtypes = [P]
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _take(lib, p, count, dtype, width=1):
    """Copy a malloc'd C array into numpy and free it."""
    n = int(count) * width
    if n:
        arr = np.ctypeslib.as_array(ctypes.cast(p, ctypes.POINTER(np.ctypeslib.as_ctypes_type(dtype))),
                                    shape=(n,)).copy()
    else:
        arr = np.zeros(0, dtype=dtype)
    lib.oracle_free(p)
    return arr


def _csr_arrays(M):
    return (np.ascontiguousarray(M.rowptr, dtype=np.int64),
            np.ascontiguousarray(M.col, dtype=np.int32),
            np.ascontiguousarray(M.val, dtype=np.int32))


def transpose(A):
    """A^T of A: SimpleNamespace(rowptr int64[m+1], read int32[nnz], pos
    int32[nnz]), rows in increasing read order.  Can be passed to overlap()
    by several threads at once (it is only read)."""
    lib = _load()
    rp, ci, va = _csr_arrays(A)
    t_rp = np.zeros(A.ncols + 1, np.int64)
    t_read = np.zeros(ci.size, np.int32)
    t_pos = np.zeros(ci.size, np.int32)
    lib.oracle_transpose(A.nrows, A.ncols, _ptr(rp), _ptr(ci), _ptr(va), _ptr(t_rp), _ptr(t_read),
                         _ptr(t_pos))
    return SimpleNamespace(rowptr=t_rp, read=t_read, pos=t_pos)


def overlap(A, min_shared: int = 1, rows=None, at=None):
    """C = A A^T over the overlap semiring.  rows: optional row subset
    (the result then has len(rows) rows, in that order).  at: A^T from
    transpose(A) (else the call builds its own)."""
    lib = _load()
    rp, ci, va = _csr_arrays(A)
    if rows is None:
        sel, nsel, nout = None, -1, A.nrows
    else:
        sel = np.ascontiguousarray(rows, dtype=np.int64)
        nsel = nout = sel.size
    out_rp = np.zeros(nout + 1, np.int64)
    pc, pn, ps = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
    nnz = ctypes.c_int64()
    if at is None:
        lib.oracle_overlap_rows(A.nrows, A.ncols, _ptr(rp), _ptr(ci), _ptr(va), int(min_shared),
                                _ptr(sel) if sel is not None else None, nsel, _ptr(out_rp),
                                ctypes.byref(pc), ctypes.byref(pn), ctypes.byref(ps),
                                ctypes.byref(nnz))
    else:
        lib.oracle_overlap_rows_t(A.nrows, A.ncols, _ptr(rp), _ptr(ci), _ptr(va), _ptr(at.rowptr),
                                  _ptr(at.read), _ptr(at.pos), int(min_shared),
                                  _ptr(sel) if sel is not None else None, nsel, _ptr(out_rp),
                                  ctypes.byref(pc), ctypes.byref(pn), ctypes.byref(ps),
                                  ctypes.byref(nnz))
    return SimpleNamespace(nrows=nout, ncols=A.nrows, rowptr=out_rp,
                           col=_take(lib, pc, nnz.value, np.int32),
                           count=_take(lib, pn, nnz.value, np.int32),
                           seed=_take(lib, ps, nnz.value, np.int32, 4).reshape(-1, 4))


def transitive_reduce(R, fuzz: int, variant: str = "A", rule: str = "row", with_walks=False):
    """S = TR(R).  Returns (S, iterations, nnz_trace) (plus the number of
    walks i -> k -> j enumerated over all passes if with_walks)."""
    lib = _load()
    rp, ci, va = _csr_arrays(R)
    flags = (VARIANT_B if variant == "B" else 0) | (RULE_EDGE if rule == "edge" else 0)
    out_rp = np.zeros(R.nrows + 1, np.int64)
    pc, pv = ctypes.c_void_p(), ctypes.c_void_p()
    nnz, iters, walks = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
    trace = np.zeros(4096, np.int64)
    lib.oracle_transitive_reduce(R.nrows, _ptr(rp), _ptr(ci), _ptr(va), int(fuzz), flags,
                                 _ptr(out_rp), ctypes.byref(pc), ctypes.byref(pv),
                                 ctypes.byref(nnz), ctypes.byref(iters), _ptr(trace), trace.size,
                                 ctypes.byref(walks))
    S = SimpleNamespace(nrows=R.nrows, ncols=R.nrows, rowptr=out_rp,
                        col=_take(lib, pc, nnz.value, np.int32),
                        val=_take(lib, pv, nnz.value, np.int32))
    ntr = min(iters.value + 1, trace.size)
    if with_walks:
        return S, iters.value, trace[:ntr].copy(), walks.value
    return S, iters.value, trace[:ntr].copy()


def tr_pass_marks(R, fuzz: int, variant: str = "A", rule: str = "row", rows=None):
    """One reduction pass on R as given: uint8 mark per entry (1 = transitive).
    Only rows in `rows` are examined (others stay 0)."""
    lib = _load()
    rp, ci, va = _csr_arrays(R)
    flags = (VARIANT_B if variant == "B" else 0) | (RULE_EDGE if rule == "edge" else 0)
    mark = np.zeros(ci.size, np.uint8)
    if rows is None:
        sel, nsel = None, -1
    else:
        sel = np.ascontiguousarray(rows, dtype=np.int64)
        nsel = sel.size
    lib.oracle_tr_pass_marks(R.nrows, _ptr(rp), _ptr(ci), _ptr(va), int(fuzz), flags,
                             _ptr(sel) if sel is not None else None, nsel, _ptr(mark))
    return mark


def r_from_seeds(C, read_len, k: int, min_overlap: int, max_drift: int = -1, min_density: int = 0):
    """Overlap graph R from the first seed of every off-diagonal entry of C
    (seed values (position << 1) | strand): suffix and code by the four
    overlap categories; pairs overlapping by fewer than min_overlap bases
    dropped, contained pairs kept with value 0.  max_drift >= 0: a pair is
    kept only if its second seed agrees (same orientation, offset within
    max_drift bases).  min_density > 0: a pair is kept only if it shares at
    least min_density k-mers per 10 kbp of its overlap.  Raises ValueError on
    a missing or out-of-range seed."""
    lib = _load()
    n = int(C.nrows)
    rp = np.ascontiguousarray(C.rowptr, dtype=np.int64)
    ci = np.ascontiguousarray(C.col, dtype=np.int32)
    cn = np.ascontiguousarray(C.count, dtype=np.int32)
    sd = np.ascontiguousarray(np.asarray(C.seed).reshape(-1), dtype=np.int32)
    ln = np.ascontiguousarray(read_len, dtype=np.int32)
    out_rp = np.zeros(n + 1, np.int64)
    pc, pv = ctypes.c_void_p(), ctypes.c_void_p()
    nnz = ctypes.c_int64()
    r = lib.oracle_r_from_seeds(n, _ptr(rp), _ptr(ci), _ptr(cn), _ptr(sd), _ptr(ln), int(k), int(min_overlap),
                                int(max_drift), int(min_density), _ptr(out_rp), ctypes.byref(pc),
                                ctypes.byref(pv), ctypes.byref(nnz))
    if r != 0:
        raise ValueError("a seed of C is missing or lies outside its read")
    return SimpleNamespace(nrows=n, ncols=n, rowptr=out_rp, col=_take(lib, pc, nnz.value, np.int32),
                           val=_take(lib, pv, nnz.value, np.int32))


def kmer_matrix(bases, offsets, k: int, lo: int, hi: int, strand_bit: bool = False):
    """A from the reads (k-mer counting, reliable k-mers in [lo, hi], the
    smallest position per read and k-mer; with strand_bit the values are
    (position << 1) | strand).  Columns are the reliable k-mers in the order
    of their first occurrence (first read holding the k-mer, then its
    smallest position there).  Returns (A, codes): A with nrows, ncols,
    rowptr, col, val; codes[c] = the canonical code of column c.  Raises
    ValueError on k outside [1, 31], bad bounds or a base outside 0..3."""
    lib = _load()
    b = np.ascontiguousarray(bases, dtype=np.uint8)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    n = len(off) - 1
    out_rp = np.zeros(n + 1, np.int64)
    pc, pv, pk = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
    m, nnz = ctypes.c_int64(), ctypes.c_int64()
    r = lib.oracle_kmer_matrix(n, _ptr(b), _ptr(off), int(k), int(lo), int(hi), 1 if strand_bit else 0,
                               _ptr(out_rp), ctypes.byref(pc), ctypes.byref(pv), ctypes.byref(pk),
                               ctypes.byref(m), ctypes.byref(nnz))
    if r != 0:
        raise ValueError("k outside [1, 31], bounds outside 1 <= lo <= hi, or a base outside 0..3")
    A = SimpleNamespace(nrows=n, ncols=m.value, nnz=nnz.value, rowptr=out_rp,
                        col=_take(lib, pc, nnz.value, np.int32), val=_take(lib, pv, nnz.value, np.int32))
    return A, _take(lib, pk, m.value, np.uint64)


def r_from_alignment(C, bases, offsets, k: int, match: int = 1, mismatch: int = -1, gap: int = -2,
                     xdrop: int = 25, min_score: int = 0):
    """Seed-and-extend alignment of every off-diagonal entry of C from its
    first seed (X-drop extension both ways, linear scores) and the graph R
    from the alignment ends of the pairs scoring at least min_score.
    Returns (R, score) with score[e] the score of C's entry e (0 on the
    diagonal).  Raises ValueError on a missing or out-of-range seed, a base
    outside 0..3, offsets that do not run from 0 up to len(bases) over
    C.ncols reads, a read of 2^28 bases or more, or scores outside match in
    [1, 7], mismatch in [-1024, 0], gap in [-1024, -1], xdrop in [0, 2^20]."""
    lib = _load()
    n = int(C.nrows)
    rp = np.ascontiguousarray(C.rowptr, dtype=np.int64)
    ci = np.ascontiguousarray(C.col, dtype=np.int32)
    sd = np.ascontiguousarray(np.asarray(C.seed).reshape(-1), dtype=np.int32)
    b = np.ascontiguousarray(bases, dtype=np.uint8)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    ncols = int(getattr(C, "ncols", n))
    if ncols != n or off.size != n + 1 or off[0] != 0 or off[-1] != b.size or np.any(np.diff(off) < 0):
        raise ValueError("C must be square with one offset per read plus one, from 0 to len(bases), non-decreasing")
    out_rp = np.zeros(n + 1, np.int64)
    score = np.zeros(len(ci), np.int32)
    pc, pv = ctypes.c_void_p(), ctypes.c_void_p()
    nnz = ctypes.c_int64()
    r = lib.oracle_r_from_alignment(n, _ptr(rp), _ptr(ci), _ptr(sd), _ptr(b), _ptr(off), int(k), int(match),
                                    int(mismatch), int(gap), int(xdrop), int(min_score), _ptr(out_rp),
                                    ctypes.byref(pc), ctypes.byref(pv), _ptr(score), ctypes.byref(nnz))
    if r != 0:
        raise ValueError("a seed of C is missing or outside its read, a base is outside 0..3, a read is too "
                         "long or a score is out of range")
    R = SimpleNamespace(nrows=n, ncols=n, nnz=nnz.value, rowptr=out_rp, col=_take(lib, pc, nnz.value, np.int32),
                        val=_take(lib, pv, nnz.value, np.int32))
    return R, score


def xdrop_extend(a, b, match: int = 1, mismatch: int = -1, gap: int = -2, xdrop: int = 25):
    """X-drop extension of base array a against b from their starts:
    (best score, (i, j) of the first cell reaching it)."""
    lib = _load()
    aa = np.ascontiguousarray(a, dtype=np.uint8)
    bb = np.ascontiguousarray(b, dtype=np.uint8)
    ea, eb = ctypes.c_int64(), ctypes.c_int64()
    s = lib.oracle_xdrop_extend(_ptr(aa), len(aa), _ptr(bb), len(bb), int(match), int(mismatch), int(gap),
                                int(xdrop), ctypes.byref(ea), ctypes.byref(eb))
    return int(s), (ea.value, eb.value)
