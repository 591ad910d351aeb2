"""ctypes binding of libdibella.so (include/dibella.h).

Argument marshalling only: torch tensors supply device memory (through the
library's allocator callbacks, which draw from PyTorch's caching allocator on
the current stream) and the HIP stream; every step of the computation runs
in the library's HIP kernels.  If the library is missing the import fails:
there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading
from dataclasses import dataclass
from typing import List, Optional, Sequence

import torch  # must be imported before the library so that both share one HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdibella.so")

OK, EINVAL, ENOMEM, EDEVICE, EOVERFLOW = 0, -1, -2, -3, -4
TR_VARIANT_B = 0x1
TR_RULE_EDGE = 0x2
NO_VALIDATE = 0x4
TR_USE_GRAPH = 0x8

EXPORTS = ["dibella_overlap", "dibella_transitive_reduce", "dibella_overlap_batched",
           "dibella_transitive_reduce_batched", "dibella_r_from_seeds", "dibella_overlap_graph_blocked",
           "dibella_transitive_reduce_noalloc", "dibella_kmer_matrix", "dibella_r_from_alignment",
           "dibella_last_error", "dibella_get_tuning",
           "dibella_set_tuning", "dibella_last_stats", "dibella_timing_enable",
           "dibella_timing_select", "dibella_timing_collect"]
PHASES = ["keys", "part_count", "part_scatter", "bucket_sort", "part2_count", "part2_scatter", "segments", "sym_bits",
          "sym_hash", "numeric", "esc", "tr_mark", "tr_compact", "numeric_phase", "r_from_seeds", "kmer_windows",
          "kmer_sort", "kmer_runs", "kmer_rows", "align"]
NUM_PHASES = 20


class DibellaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"dibella status {status}: {msg}")
        self.status = status


class _CSR(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("ncols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("rowptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class _OverlapOut(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("ncols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("rowptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("count", ctypes.c_void_p),
                ("seed", ctypes.c_void_p)]


class _CSROut(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("ncols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("rowptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int32) for name in (
        "sym_block", "num_block", "tr_block", "sym_first_log2", "sym_max_log2", "num_max_entries",
        "load_pct", "tr_lds_cap", "tr_graph_passes", "bits_max_words")]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class _Stats(ctypes.Structure):
    _fields_ = [("products", ctypes.c_int64), ("esc_rows", ctypes.c_int64),
                ("host_syncs", ctypes.c_int64), ("triples", ctypes.c_int64),
                ("passes", ctypes.c_int32), ("trace_len", ctypes.c_int32),
                ("nnz_trace", ctypes.c_int64 * 64), ("triples_trace", ctypes.c_int64 * 64),
                ("cells", ctypes.c_int64)]


class _Timing(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * NUM_PHASES), ("records", ctypes.c_int64 * NUM_PHASES)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    P, i32, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32
    lib.dibella_overlap.argtypes = [P, i32, P, ALLOC_FN, FREE_FN, P, P]
    lib.dibella_overlap_batched.argtypes = [P, i32, P, P, ALLOC_FN, FREE_FN, P, P]
    lib.dibella_transitive_reduce.argtypes = [P, i32, u32, P, P, ALLOC_FN, FREE_FN, P, P]
    lib.dibella_transitive_reduce_batched.argtypes = [P, i32, P, u32, P, P, ALLOC_FN, FREE_FN, P, P]
    lib.dibella_r_from_seeds.argtypes = [P, P, i32, i32, i32, i32, P, ALLOC_FN, FREE_FN, P, P]
    lib.dibella_overlap_graph_blocked.argtypes = [P, i32, P, i32, i32, i32, i32, ctypes.c_int64, P, P, ALLOC_FN,
                                                  FREE_FN, P, P]
    lib.dibella_transitive_reduce_noalloc.argtypes = [P, i32, u32, P, P, P, ctypes.c_int64, P, P, P]
    lib.dibella_r_from_alignment.argtypes = [P, P, ctypes.c_int64, P, i32, i32, i32, i32, i32, i32, u32, P, P,
                                             ALLOC_FN, FREE_FN, P, P]
    lib.dibella_kmer_matrix.argtypes = [P, P, ctypes.c_int64, ctypes.c_int64, i32, i32, i32, u32, P, P, ALLOC_FN,
                                        FREE_FN, P, P]
    for f in EXPORTS:
        getattr(lib, f).restype = ctypes.c_int
    lib.dibella_last_error.restype = ctypes.c_char_p
    lib.dibella_last_error.argtypes = []
    lib.dibella_get_tuning.argtypes = [P]
    lib.dibella_set_tuning.argtypes = [P]
    lib.dibella_last_stats.argtypes = [P]
    lib.dibella_timing_enable.argtypes = [ctypes.c_int]
    lib.dibella_timing_select.argtypes = [ctypes.c_uint32]
    lib.dibella_timing_collect.argtypes = [P]
    return lib


_lib: Optional[ctypes.CDLL] = None
_lock = threading.Lock()


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        with _lock:
            if _lib is None:
                _lib = load_library()
    return _lib


# ---------------------------------------------------------------------------
# Allocator: every byte the library asks for is a torch uint8 tensor on the
# current device and stream.  Live blocks are kept per call in a registry so
# that outputs can be handed back as tensors.
# ---------------------------------------------------------------------------
class _Allocations:
    def __init__(self, device: torch.device):
        self.device = device
        self.live = {}

    def alloc(self, nbytes: int, _ctx) -> int:
        try:
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        except Exception:  # out of memory: the library reports DIBELLA_ENOMEM
            return 0
        p = t.data_ptr()
        self.live[p] = t
        return p

    def free(self, p: int, _ctx) -> None:
        self.live.pop(p, None)

    def take(self, p: Optional[int], dtype: torch.dtype, count: int) -> torch.Tensor:
        if not p or count == 0:
            return torch.empty(0, dtype=dtype, device=self.device)
        t = self.live.pop(p)
        return t.view(dtype)[:count]


class _Call:
    """Callbacks bound to one call (ctypes keeps no reference itself)."""

    def __init__(self, device: torch.device):
        self.mem = _Allocations(device)
        self.alloc_cb = ALLOC_FN(self.mem.alloc)
        self.free_cb = FREE_FN(self.mem.free)


_tls = threading.local()


def _call_for(device: torch.device) -> _Call:
    """The calling thread's callbacks for `device`, with an empty registry
    (calls on one thread run one after another, so they can share them)."""
    cache = getattr(_tls, "calls", None)
    if cache is None:
        cache = _tls.calls = {}
    c = cache.get(device)
    if c is None:
        c = cache[device] = _Call(device)
    c.mem.live.clear()
    return c


def _stream_handle(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _check(status: int) -> None:
    if status != OK:
        raise DibellaError(status, lib().dibella_last_error().decode())


# ---------------------------------------------------------------------------
# Public data holders
# ---------------------------------------------------------------------------
@dataclass
class CSRTensors:
    """CSR on the device: rowptr int64[n+1], col int32, val int32."""
    nrows: int
    ncols: int
    rowptr: torch.Tensor
    col: torch.Tensor
    val: torch.Tensor

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    @classmethod
    def from_numpy(cls, M, device="cuda"):
        return cls(int(M.nrows), int(M.ncols),
                   torch.as_tensor(M.rowptr, dtype=torch.int64).to(device),
                   torch.as_tensor(M.col, dtype=torch.int32).to(device),
                   torch.as_tensor(M.val, dtype=torch.int32).to(device))


@dataclass
class OverlapCSR:
    nrows: int
    ncols: int
    rowptr: torch.Tensor   # int64[n+1]
    col: torch.Tensor      # int32[nnz]
    count: torch.Tensor    # int32[nnz]
    seed: torch.Tensor     # int32[nnz, 4]

    @property
    def nnz(self) -> int:
        return int(self.col.numel())


def _csr_struct(M: CSRTensors) -> _CSR:
    for name, t, dt in (("rowptr", M.rowptr, torch.int64), ("col", M.col, torch.int32),
                        ("val", M.val, torch.int32)):
        if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous {dt} device tensor")
    return _CSR(M.nrows, M.ncols, M.nnz, M.rowptr.data_ptr(),
                M.col.data_ptr() if M.nnz else None, M.val.data_ptr() if M.nnz else None)


def _device_of(mats: Sequence[CSRTensors]) -> torch.device:
    return mats[0].rowptr.device if mats else torch.device("cuda", torch.cuda.current_device())


def overlap_batched(As: Sequence[CSRTensors], min_shared) -> List[OverlapCSR]:
    """C_s = A_s A_s^T for every set, in one set of launches."""
    n = len(As)
    if isinstance(min_shared, int):
        min_shared = [min_shared] * n
    dev = _device_of(As)
    call = _call_for(dev)
    ins = (_CSR * max(n, 1))(*[_csr_struct(a) for a in As])
    outs = (_OverlapOut * max(n, 1))()
    ms = (ctypes.c_int32 * max(n, 1))(*min_shared)
    with torch.cuda.device(dev):
        st = lib().dibella_overlap_batched(ins, n, ms, outs, call.alloc_cb, call.free_cb, None,
                                           _stream_handle(dev))
    _check(st)
    res = []
    for s in range(n):
        o = outs[s]
        res.append(OverlapCSR(o.nrows, o.ncols,
                              call.mem.take(o.rowptr, torch.int64, o.nrows + 1),
                              call.mem.take(o.col, torch.int32, o.nnz),
                              call.mem.take(o.count, torch.int32, o.nnz),
                              call.mem.take(o.seed, torch.int32, 4 * o.nnz).view(-1, 4)))
    return res


def overlap(A: CSRTensors, min_shared: int = 1) -> OverlapCSR:
    """C = A A^T over the overlap semiring (count + two seeds)."""
    dev = _device_of([A])
    call = _call_for(dev)
    a = _csr_struct(A)
    o = _OverlapOut()
    with torch.cuda.device(dev):
        st = lib().dibella_overlap(ctypes.byref(a), int(min_shared), ctypes.byref(o), call.alloc_cb,
                                   call.free_cb, None, _stream_handle(dev))
    _check(st)
    return OverlapCSR(o.nrows, o.ncols, call.mem.take(o.rowptr, torch.int64, o.nrows + 1),
                      call.mem.take(o.col, torch.int32, o.nnz),
                      call.mem.take(o.count, torch.int32, o.nnz),
                      call.mem.take(o.seed, torch.int32, 4 * o.nnz).view(-1, 4))


def tr_flags(variant: str = "A", rule: str = "row", graph: bool = False, max_passes: int = 0,
             validate: bool = True) -> int:
    f = (TR_VARIANT_B if variant == "B" else 0) | (TR_RULE_EDGE if rule == "edge" else 0)
    f |= (TR_USE_GRAPH if graph else 0) | (0 if validate else NO_VALIDATE)
    return f | ((int(max_passes) & 0xFFFF) << 16)


def transitive_reduce_batched(Rs: Sequence[CSRTensors], fuzz, variant="A", rule="row", graph=False,
                              max_passes=0):
    """S_s = TR(R_s) for every set in one set of launches.  Returns (list of
    S, list of pass counts)."""
    n = len(Rs)
    if isinstance(fuzz, int):
        fuzz = [fuzz] * n
    dev = _device_of(Rs)
    call = _call_for(dev)
    ins = (_CSR * max(n, 1))(*[_csr_struct(r) for r in Rs])
    outs = (_CSROut * max(n, 1))()
    fz = (ctypes.c_int32 * max(n, 1))(*fuzz)
    its = (ctypes.c_int32 * max(n, 1))()
    with torch.cuda.device(dev):
        st = lib().dibella_transitive_reduce_batched(
            ins, n, fz, tr_flags(variant, rule, graph, max_passes), outs, its, call.alloc_cb,
            call.free_cb, None, _stream_handle(dev))
    _check(st)
    res = []
    for s in range(n):
        o = outs[s]
        res.append(CSRTensors(o.nrows, o.ncols, call.mem.take(o.rowptr, torch.int64, o.nrows + 1),
                              call.mem.take(o.col, torch.int32, o.nnz),
                              call.mem.take(o.val, torch.int32, o.nnz)))
    return res, [int(its[s]) for s in range(n)]


def transitive_reduce(R: CSRTensors, fuzz: int, variant="A", rule="row", graph=False, max_passes=0,
                      validate=True):
    """S = TR(R).  Returns (S, passes executed)."""
    dev = _device_of([R])
    call = _call_for(dev)
    r = _csr_struct(R)
    o = _CSROut()
    it = ctypes.c_int32()
    with torch.cuda.device(dev):
        st = lib().dibella_transitive_reduce(
            ctypes.byref(r), int(fuzz), tr_flags(variant, rule, graph, max_passes, validate),
            ctypes.byref(o), ctypes.byref(it), call.alloc_cb, call.free_cb, None, _stream_handle(dev))
    _check(st)
    S = CSRTensors(o.nrows, o.ncols, call.mem.take(o.rowptr, torch.int64, o.nrows + 1),
                   call.mem.take(o.col, torch.int32, o.nnz), call.mem.take(o.val, torch.int32, o.nnz))
    return S, int(it.value)


def r_from_seeds(C: OverlapCSR, read_len: torch.Tensor, k: int, min_overlap: int,
                 max_drift: int = -1, min_density: int = 0) -> CSRTensors:
    """Overlap graph R from the first seed of every off-diagonal entry of C
    (A's values being (position << 1) | strand): the suffix and orientation
    code by the four overlap categories, pairs overlapping by fewer than
    min_overlap bases dropped, contained pairs kept with value 0.  With
    max_drift >= 0 the second seed must agree (same orientation, offset
    within max_drift bases); with min_density > 0 the pair must share at
    least min_density k-mers per 10 kbp of its overlap."""
    dev = C.rowptr.device
    if read_len.dtype != torch.int32 or not read_len.is_cuda or not read_len.is_contiguous():
        raise TypeError("read_len must be a contiguous int32 device tensor")
    if read_len.numel() != C.nrows:
        raise ValueError("read_len must hold one length per row of C")
    call = _call_for(dev)
    for name, t, dt in (("rowptr", C.rowptr, torch.int64), ("col", C.col, torch.int32),
                        ("count", C.count, torch.int32), ("seed", C.seed, torch.int32)):
        if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
            raise TypeError(f"C.{name} must be a contiguous {dt} device tensor")
    c = _OverlapOut(C.nrows, C.ncols, C.nnz, C.rowptr.data_ptr(), C.col.data_ptr() if C.nnz else None,
                    C.count.data_ptr() if C.nnz else None, C.seed.data_ptr() if C.nnz else None)
    o = _CSROut()
    with torch.cuda.device(dev):
        st = lib().dibella_r_from_seeds(ctypes.byref(c), read_len.data_ptr() if C.nrows else None, int(k),
                                        int(min_overlap), int(max_drift), int(min_density), ctypes.byref(o),
                                        call.alloc_cb, call.free_cb, None, _stream_handle(dev))
    _check(st)
    return CSRTensors(o.nrows, o.ncols, call.mem.take(o.rowptr, torch.int64, o.nrows + 1),
                      call.mem.take(o.col, torch.int32, o.nnz), call.mem.take(o.val, torch.int32, o.nnz))


def overlap_graph_blocked(A: CSRTensors, min_shared: int, read_len: torch.Tensor, k: int, min_overlap: int,
                          max_drift: int = -1, min_density: int = 0, block_rows: int = 1 << 30):
    """The overlap graph R = r_from_seeds(overlap(A, min_shared), ...) with C
    formed block_rows reads at a time (A^T built once; each block's rows of
    C turned into R and released before the next block).  Returns (R, number
    of blocks)."""
    dev = _device_of([A])
    if read_len.dtype != torch.int32 or not read_len.is_cuda or not read_len.is_contiguous():
        raise TypeError("read_len must be a contiguous int32 device tensor")
    if read_len.numel() != A.nrows:
        raise ValueError("read_len must hold one length per row of A")
    call = _call_for(dev)
    a = _csr_struct(A)
    o = _CSROut()
    nb = ctypes.c_int32(0)
    with torch.cuda.device(dev):
        st = lib().dibella_overlap_graph_blocked(ctypes.byref(a), int(min_shared),
                                                 read_len.data_ptr() if A.nrows else None, int(k), int(min_overlap),
                                                 int(max_drift), int(min_density), int(block_rows), ctypes.byref(o),
                                                 ctypes.byref(nb), call.alloc_cb, call.free_cb, None,
                                                 _stream_handle(dev))
    _check(st)
    R = CSRTensors(o.nrows, o.ncols, call.mem.take(o.rowptr, torch.int64, o.nrows + 1),
                   call.mem.take(o.col, torch.int32, o.nnz), call.mem.take(o.val, torch.int32, o.nnz))
    return R, nb.value


KMER_STRAND = 0x1


def kmer_matrix(bases: torch.Tensor, offsets: torch.Tensor, k: int, lo: int, hi: int, strand_bit: bool = False):
    """A from the reads on the device: bases uint8 (A0 C1 G2 T3, reads back
    to back), offsets int64[n + 1].  Reliable k-mers (frequency over all
    windows in [lo, hi]) are the columns in the order of their first
    occurrence (first read holding the k-mer, then its smallest position
    there); values are the smallest position per read and k-mer (with
    strand_bit: (position << 1) | strand).  Returns (A, codes): codes[c] =
    the canonical code of column c (int64 tensor)."""
    if bases.dtype != torch.uint8 or not bases.is_cuda or not bases.is_contiguous():
        raise TypeError("bases must be a contiguous uint8 device tensor")
    if offsets.dtype != torch.int64 or not offsets.is_cuda or not offsets.is_contiguous() or offsets.numel() < 1:
        raise TypeError("offsets must be a contiguous int64 device tensor of n + 1 entries")
    dev = bases.device
    call = _call_for(dev)
    n = offsets.numel() - 1
    o = _CSROut()
    codes = ctypes.c_void_p()
    with torch.cuda.device(dev):
        st = lib().dibella_kmer_matrix(bases.data_ptr() if bases.numel() else None, offsets.data_ptr(), n,
                                       bases.numel(), int(k), int(lo), int(hi), KMER_STRAND if strand_bit else 0,
                                       ctypes.byref(o), ctypes.byref(codes), call.alloc_cb, call.free_cb, None,
                                       _stream_handle(dev))
    _check(st)
    A = CSRTensors(o.nrows, o.ncols, call.mem.take(o.rowptr, torch.int64, o.nrows + 1),
                   call.mem.take(o.col, torch.int32, o.nnz), call.mem.take(o.val, torch.int32, o.nnz))
    return A, call.mem.take(codes.value, torch.int64, o.ncols)


ALIGN_GROUPS = {None: 0, 16: 0x1, 32: 0x2, 64: 0x3}


def r_from_alignment(C: OverlapCSR, bases: torch.Tensor, offsets: torch.Tensor, k: int, match: int = 1,
                     mismatch: int = -1, gap: int = -2, xdrop: int = 25, min_score: int = 0,
                     group: int = None, with_score: bool = False):
    """Overlap graph R from a seed-and-extend alignment of every pair of C
    (A's values being (position << 1) | strand): X-drop extension both ways
    from the first seed, read j reverse complemented when the strands
    differ; pairs scoring below min_score dropped; the suffix and
    orientation code from the alignment ends, contained pairs kept with
    value 0.  bases uint8 (A0 C1 G2 T3, reads back to back), offsets
    int64[n + 1].  group: lanes per extension of the general kernel over
    every extension (16, 32, 64; None = the register-band fast path with
    lanes chosen from the scores, the general kernel redoing extensions
    whose band outgrows it; the result is the same).  Returns R, or (R,
    score) with the int32 score of every entry of C (0 on the diagonal)."""
    dev = C.rowptr.device
    if bases.dtype != torch.uint8 or not bases.is_cuda or not bases.is_contiguous():
        raise TypeError("bases must be a contiguous uint8 device tensor")
    if offsets.dtype != torch.int64 or not offsets.is_cuda or not offsets.is_contiguous():
        raise TypeError("offsets must be a contiguous int64 device tensor")
    if offsets.numel() != C.nrows + 1:
        raise ValueError("offsets must hold one entry per row of C plus one")
    if group not in ALIGN_GROUPS:
        raise ValueError("group must be 16, 32, 64 or None")
    call = _call_for(dev)
    for name, t, dt in (("rowptr", C.rowptr, torch.int64), ("col", C.col, torch.int32),
                        ("seed", C.seed, torch.int32)):
        if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
            raise TypeError(f"C.{name} must be a contiguous {dt} device tensor")
    c = _OverlapOut(C.nrows, C.ncols, C.nnz, C.rowptr.data_ptr(), C.col.data_ptr() if C.nnz else None,
                    C.count.data_ptr() if C.nnz else None, C.seed.data_ptr() if C.nnz else None)
    o = _CSROut()
    sc = ctypes.c_void_p()
    with torch.cuda.device(dev):
        st = lib().dibella_r_from_alignment(ctypes.byref(c), bases.data_ptr() if bases.numel() else None,
                                            bases.numel(), offsets.data_ptr(), int(k), int(match), int(mismatch),
                                            int(gap), int(xdrop), int(min_score), ALIGN_GROUPS[group],
                                            ctypes.byref(o), ctypes.byref(sc) if with_score else None,
                                            call.alloc_cb, call.free_cb, None, _stream_handle(dev))
    _check(st)
    R = CSRTensors(o.nrows, o.ncols, call.mem.take(o.rowptr, torch.int64, o.nrows + 1),
                   call.mem.take(o.col, torch.int32, o.nnz), call.mem.take(o.val, torch.int32, o.nnz))
    if with_score:
        return R, call.mem.take(sc.value, torch.int32, C.nnz)
    return R


def last_stats() -> dict:
    s = _Stats()
    _check(lib().dibella_last_stats(ctypes.byref(s)))
    n = s.trace_len
    return {"products": s.products, "esc_rows": s.esc_rows, "host_syncs": s.host_syncs,
            "triples": s.triples, "passes": s.passes,
            "nnz_trace": [s.nnz_trace[i] for i in range(n)],
            "triples_trace": [s.triples_trace[i] for i in range(max(0, min(s.passes, 64)))],
            "cells": s.cells}


def get_tuning() -> dict:
    t = Tuning()
    _check(lib().dibella_get_tuning(ctypes.byref(t)))
    return t.as_dict()


def set_tuning(**kw) -> dict:
    cur = get_tuning()
    cur.update(kw)
    t = Tuning(**cur)
    _check(lib().dibella_set_tuning(ctypes.byref(t)))
    return cur


def timing_enable(on: bool = True) -> None:
    """Record HIP events around the main kernels of later calls on this thread."""
    _check(lib().dibella_timing_enable(1 if on else 0))


def timing_select(labels=None) -> None:
    """Record only these labels (names of PHASES) from now on; None = all."""
    if labels is None:
        mask = (1 << len(PHASES)) - 1
    else:
        mask = 0
        for name in labels:
            mask |= 1 << PHASES.index(name)
    _check(lib().dibella_timing_select(mask))


def timing_collect() -> dict:
    """{phase: (milliseconds summed, records)} since enabling / the last collect."""
    t = _Timing()
    _check(lib().dibella_timing_collect(ctypes.byref(t)))
    return {name: (t.ms[i], int(t.records[i])) for i, name in enumerate(PHASES)}
