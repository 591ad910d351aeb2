"""Host-side checks of the HIP library that need no GPU: it loads, exports
every symbol the header declares, and its argument checks and tuning
interface behave."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dibella.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(dibella_[a-z_]+)\s*\(", text)) - {"dibella_alloc_fn", "dibella_free_fn"})


@pytest.fixture(scope="module")
def lib():
    from paper_2010_10055_amd import _lib
    return _lib.lib()


def test_library_exports_every_declared_symbol(lib):
    names = _declared()
    assert "dibella_overlap" in names and "dibella_transitive_reduce" in names
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_header():
    from paper_2010_10055_amd import _lib
    assert sorted(_lib.EXPORTS) == _declared()


def test_null_arguments_rejected_without_gpu(lib):
    from paper_2010_10055_amd import _lib
    st = lib.dibella_overlap(None, 1, None, _lib.ALLOC_FN(0), _lib.FREE_FN(0), None, None)
    assert st == _lib.EINVAL
    assert b"bad arguments" in lib.dibella_last_error()
    it = ctypes.c_int32()
    st = lib.dibella_transitive_reduce(None, 0, 0, None, ctypes.byref(it), _lib.ALLOC_FN(0),
                                       _lib.FREE_FN(0), None, None)
    assert st == _lib.EINVAL


def test_zero_sets_is_a_no_op(lib):
    from paper_2010_10055_amd import _lib
    dummy = (_lib._CSR * 1)()
    out = (_lib._OverlapOut * 1)()
    ms = (ctypes.c_int32 * 1)(1)
    assert lib.dibella_overlap_batched(dummy, 0, ms, out, _lib.ALLOC_FN(0), _lib.FREE_FN(0), None,
                                       None) == _lib.OK


def test_tuning_roundtrip_and_range_checks():
    import paper_2010_10055_amd as pkg
    old = pkg.get_tuning()
    try:
        new = pkg.set_tuning(num_block=128, tr_lds_cap=2048)
        assert pkg.get_tuning() == new
        for bad in ({"sym_block": 96}, {"num_max_entries": 9000}, {"tr_graph_passes": 0},
                    {"sym_max_log2": 15}, {"load_pct": 90}, {"sym_first_log2": 14}):
            with pytest.raises(pkg.DibellaError):
                pkg.set_tuning(**bad)
        assert pkg.get_tuning() == new
    finally:
        pkg.set_tuning(**old)


def test_timing_label_selection_range(lib):
    from paper_2010_10055_amd import _lib
    assert lib.dibella_timing_select(1 << _lib.NUM_PHASES) == _lib.EINVAL   # label bits beyond the labels
    assert lib.dibella_timing_select(0xFFFFFFFF) == _lib.EINVAL
    assert lib.dibella_timing_select(0) == _lib.OK
    _lib.timing_select(["numeric_phase", "tr_mark"])
    with pytest.raises(ValueError):
        _lib.timing_select(["no_such_label"])
    _lib.timing_select(None)
    assert lib.dibella_timing_select((1 << _lib.NUM_PHASES) - 1) == _lib.OK


def test_timing_labels_match_the_header():
    from paper_2010_10055_amd import _lib
    text = open(os.path.join(ROOT, "include", "dibella.h")).read()
    block = text[text.index("Kernel timing with HIP events"):text.index("#define DIBELLA_NUM_PHASES")]
    labels = dict((int(n), name) for n, name in re.findall(r"^\s*\*\s+(\d+)\s+(\w+)", block, re.M))
    assert [labels[i] for i in range(len(labels))] == _lib.PHASES
    assert len(_lib.PHASES) <= int(re.search(r"#define DIBELLA_NUM_PHASES (\d+)", text).group(1))


def test_stats_struct_matches_the_header(lib):
    """The binding's mirror of dibella_stats has the header's fields in the
    header's order, with the same widths, and the library fills a struct of
    exactly that size (the last field is read back after a reset)."""
    from paper_2010_10055_amd import _lib
    text = open(HEADER).read()
    body = text[text.index("/* Counters of the last call"):text.index("} dibella_stats;")]
    body = body[body.index("typedef struct {") + len("typedef struct {"):]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"(int64_t|int32_t)\s+(\w+)(?:\[(\d+)\])?;", body)
    width = {"int64_t": ctypes.c_int64, "int32_t": ctypes.c_int32}
    want = [(name, width[t] * int(n) if n else width[t]) for t, name, n in fields]
    got = list(_lib._Stats._fields_)
    assert [f for f, _ in got] == [f for f, _ in want]
    for (_, a), (_, b) in zip(got, want):
        assert ctypes.sizeof(a) == ctypes.sizeof(b)
    s = _lib._Stats()
    s.cells = 12345
    assert lib.dibella_last_stats(ctypes.byref(s)) == 0
    assert s.cells == 0          # the thread's counters start at zero
