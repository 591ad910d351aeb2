"""Serving scheduler on the CPU: a fake executor (the oracle) and a virtual
clock force arrivals, batching, admission by footprint, rejection of an
oversized job and a failing job, without a GPU."""
import numpy as np
import pytest

import oracle
from paper_2010_10055_amd import serve, synth


def _fake(clock, per_job_s=0.010, overhead_s=0.002, fail_ids=()):
    calls = []

    def execute(batch):
        calls.append([j.jid for j in batch])
        if any(j.jid in fail_ids for j in batch):
            clock.advance(overhead_s)
            raise RuntimeError("bad job in batch")
        # batched work overlaps: the step costs its largest job plus overhead
        clock.advance(overhead_s + per_job_s * max(1.0, 0.5 * len(batch)))
        return [oracle.overlap(j.payload, 1) for j in batch]

    return execute, calls


def _jobs(rate, count, seed=0, footprint=100):
    rng = np.random.default_rng(seed)
    times = serve.poisson_arrivals(rng, count, rate)
    out = []
    for q in range(count):
        A = synth.random_a(np.random.default_rng(100 + q), 20, 40, 0.1)
        out.append(serve.Job(q, float(times[q]), A, footprint))
    return out


def test_every_job_completes_and_results_match_solo():
    clock = serve.VirtualClock()
    execute, calls = _fake(clock)
    jobs = _jobs(rate=400.0, count=60)
    done = serve.serve(jobs, execute, clock, hbm_budget=10_000, max_batch=16)
    assert sorted(d.jid for d in done) == list(range(60))
    by = {d.jid: d for d in done}
    for j in jobs:
        d = by[j.jid]
        assert d.error is None and d.finish >= d.start >= j.arrival
        solo = oracle.overlap(j.payload, 1)
        assert np.array_equal(d.result.col, solo.col) and np.array_equal(d.result.seed, solo.seed)
    # arrivals outpace single-job service: jobs were batched
    assert max(len(c) for c in calls) > 1


def test_admission_respects_the_budget_and_rejects_oversized_jobs():
    clock = serve.VirtualClock()
    execute, calls = _fake(clock)
    jobs = _jobs(rate=1000.0, count=30, footprint=300)
    jobs[7] = serve.Job(7, jobs[7].arrival, jobs[7].payload, footprint=5000)
    done = serve.serve(jobs, execute, clock, hbm_budget=1000, max_batch=64)
    for c in calls:
        assert len(c) <= 3   # 3 x 300 <= 1000 < 4 x 300
    bad = [d for d in done if d.error]
    assert [d.jid for d in bad] == [7]
    assert sum(1 for d in done if d.error is None) == 29


def test_a_failing_job_fails_alone():
    clock = serve.VirtualClock()
    execute, calls = _fake(clock, fail_ids=(5,))
    jobs = _jobs(rate=800.0, count=20)
    done = serve.serve(jobs, execute, clock, hbm_budget=10_000, max_batch=8)
    errs = {d.jid for d in done if d.error}
    assert errs == {5}
    assert len(done) == 20


def test_fifo_runs_in_arrival_order_one_at_a_time():
    clock = serve.VirtualClock()
    execute, calls = _fake(clock)
    jobs = _jobs(rate=50.0, count=15)
    done = serve.serve(jobs, execute, clock, hbm_budget=10_000, max_batch=1)
    assert [c[0] for c in calls] == list(range(15)) and all(len(c) == 1 for c in calls)
    s = serve.summarize(done, clock.now())
    assert s["ok"] == 15 and s["p99_ms"] >= s["p50_ms"] > 0


def test_batching_beats_fifo_under_load():
    jobs = _jobs(rate=300.0, count=80)
    res = {}
    for mb in (1, 32):
        clock = serve.VirtualClock()
        execute, _ = _fake(clock)
        done = serve.serve(jobs, execute, clock, hbm_budget=100_000, max_batch=mb)
        res[mb] = serve.summarize(done, clock.now())
    assert res[32]["p99_ms"] < res[1]["p99_ms"]
    assert res[32]["jobs_per_s"] > res[1]["jobs_per_s"]


def test_footprint_estimate_grows_with_size():
    small = serve.footprint_bytes(200, 5e4, 1.2e5, 1, 3e3)
    big = serve.footprint_bytes(3e4, 4e7, 1.5e8, 2, 1.6e6)
    assert 0 < small < big
