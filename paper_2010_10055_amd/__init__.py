"""MI355X (gfx950) library for the two semiring sparse products of diBELLA 2D:
the candidate overlap matrix C = A A^T and the transitive reduction of the
overlap graph.  The computation lives in libdibella.so (hand-written HIP);
this package is its Python binding plus the synthetic workload generator.
"""
from ._lib import (CSRTensors, DibellaError, OverlapCSR, get_tuning, last_stats, overlap,  # noqa: F401
                   kmer_matrix, overlap_batched, overlap_graph_blocked, r_from_alignment, r_from_seeds, set_tuning, timing_collect, timing_enable,
                   timing_select, transitive_reduce, transitive_reduce_batched)

__all__ = ["CSRTensors", "OverlapCSR", "DibellaError", "overlap", "overlap_batched", "r_from_seeds",
           "r_from_alignment",
           "overlap_graph_blocked", "kmer_matrix",
           "transitive_reduce", "transitive_reduce_batched", "last_stats", "get_tuning", "set_tuning",
           "timing_enable", "timing_select", "timing_collect"]
