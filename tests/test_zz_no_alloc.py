"""The reduction entry point that allocates nothing
(dibella_transitive_reduce_noalloc), called through the C ABI with ctypes,
against dibella_transitive_reduce on the same inputs: two calls in a row,
the second on a smaller input (the static scratch keeps the first call's
contents), plus its argument checks."""
import ctypes

import numpy as np
import pytest

from paper_2010_10055_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def db():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_10055_amd as pkg
    return pkg


def _noalloc(pkg, R, fuzz, flags=0, capacity=None):
    from paper_2010_10055_amd import _lib
    dev = R.rowptr.device
    cap = R.nnz if capacity is None else capacity
    rp = torch.full((R.nrows + 1,), -7, dtype=torch.int64, device=dev)
    col = torch.full((max(cap, 1),), -7, dtype=torch.int32, device=dev)
    val = torch.full((max(cap, 1),), -7, dtype=torch.int32, device=dev)
    nnz, it = ctypes.c_int64(-1), ctypes.c_int32(-1)
    r = _lib._csr_struct(R)
    torch.cuda.synchronize()
    st = _lib.lib().dibella_transitive_reduce_noalloc(
        ctypes.byref(r), int(fuzz), int(flags), rp.data_ptr(), col.data_ptr(), val.data_ptr(), int(cap),
        ctypes.byref(nnz), ctypes.byref(it), torch.cuda.current_stream(dev).cuda_stream)
    torch.cuda.synchronize()
    return st, rp, col[:max(nnz.value, 0)], val[:max(nnz.value, 0)], it.value


def _check_same(pkg, R, fuzz, variant="A", rule="row"):
    flags = pkg._lib.tr_flags(variant, rule)
    st, rp, col, val, it = _noalloc(pkg, R, fuzz, flags)
    assert st == 0, pkg._lib.lib().dibella_last_error().decode()
    S, it0 = pkg.transitive_reduce(R, fuzz, variant=variant, rule=rule)
    torch.cuda.synchronize()
    assert it == it0
    assert torch.equal(rp, S.rowptr) and torch.equal(col, S.col) and torch.equal(val, S.val)
    return S.nnz


def test_noalloc_equals_allocating_call_twice_second_smaller(db):
    big = synth.make_workload("tiny", seed=1000)
    R1 = db.CSRTensors.from_numpy(big.R, "cuda:0")
    rng = np.random.default_rng(5)
    small = synth.perturb_graph(rng, synth.random_r(rng, 60, 0.08, max_overhang=300), false_edges=20)
    R2 = db.CSRTensors.from_numpy(small, "cuda:0")
    print(f"noalloc: R1 {R1.nrows} rows {R1.nnz} entries, R2 {R2.nrows} rows {R2.nnz} entries", flush=True)
    assert R2.nnz < R1.nnz and R2.nrows < R1.nrows
    assert _check_same(db, R1, big.fuzz) > 0
    assert _check_same(db, R2, 150, variant="B") > 0
    assert _check_same(db, R1, big.fuzz, rule="edge") > 0


def test_noalloc_mid_size_reduction(db):
    """A larger R (the batch workload's first set), still within the scratch."""
    w = synth.make_workload("batchset", seed=4002)
    R = db.CSRTensors.from_numpy(w.R, "cuda:0")
    print(f"noalloc: {R.nrows} rows {R.nnz} entries", flush=True)
    _check_same(db, R, w.fuzz)


def test_noalloc_argument_checks(db):
    w = synth.make_workload("tiny", seed=1001)
    R = db.CSRTensors.from_numpy(w.R, "cuda:0")
    st, *_ = _noalloc(db, R, w.fuzz, capacity=R.nnz - 1)
    assert st == -1
    st, *_ = _noalloc(db, R, w.fuzz, flags=db._lib.TR_USE_GRAPH)
    assert st == -1
    # beyond the 64 MiB of workspace: rejected before any work (no kernel reads the fake arrays)
    n = 2_000_000
    fake = db.CSRTensors(n, n, torch.zeros(n + 1, dtype=torch.int64, device="cuda:0"),
                         torch.zeros(4_000_000, dtype=torch.int32, device="cuda:0"),
                         torch.zeros(4_000_000, dtype=torch.int32, device="cuda:0"))
    st, *_ = _noalloc(db, fake, 10)
    assert st == -1
    assert "maximum" in db._lib.lib().dibella_last_error().decode()
    # a malformed R fails cleanly and the next call works
    bad = db.CSRTensors(R.nrows, R.ncols, R.rowptr, R.col.clone(), R.val)
    bad.col[0] = R.nrows + 5
    st, *_ = _noalloc(db, bad, w.fuzz)
    assert st == -1
    _check_same(db, R, w.fuzz)
