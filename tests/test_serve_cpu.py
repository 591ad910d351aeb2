"""Serving scheduler on the CPU: a virtual-time executor (running the oracle)
and a virtual clock force arrivals, overlapping admission, admission by
footprint, rejection of an oversized job and a failing job, without a GPU."""
import numpy as np

import oracle
from paper_2010_10055_amd import serve, synth


def _executor(clock, base_s=0.010, share=0.3, fail_ids=()):
    """A job takes base_s, stretched by `share` for every job already running
    when it starts (jobs sharing the device slow each other down)."""
    return serve.VirtualExecutor(clock, lambda A: oracle.overlap(A, 1),
                                 lambda job, running: base_s * (1.0 + share * running), fail_ids)


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
    ex = _executor(clock)
    jobs = _jobs(rate=400.0, count=60)
    st = {}
    done = serve.serve(jobs, ex, clock, hbm_budget=10_000, slots=4, stats=st)
    assert sorted(d.jid for d in done) == list(range(60))
    by = {d.jid: d for d in done}
    for j in jobs:
        d = by[j.jid]
        assert d.error is None and d.finish >= d.start >= j.arrival
        solo = oracle.overlap(j.payload, 1)
        assert np.array_equal(d.result.col, solo.col) and np.array_equal(d.result.seed, solo.seed)
    # arrivals outpace single-job service: jobs ran side by side
    assert st["peak_running"] > 1 and st["peak_running"] <= 4


def test_a_job_arriving_while_others_run_starts_before_they_finish():
    """Continuous admission: a slot that is free takes an arriving job at
    once, it does not wait for the running jobs to end."""
    clock = serve.VirtualClock()
    ex = _executor(clock, base_s=0.050, share=0.0)
    jobs = [serve.Job(0, 0.0, synth.random_a(np.random.default_rng(1), 10, 20, 0.2), 1),
            serve.Job(1, 0.010, synth.random_a(np.random.default_rng(2), 10, 20, 0.2), 1)]
    done = {d.jid: d for d in serve.serve(jobs, ex, clock, hbm_budget=100, slots=2)}
    assert done[1].start == 0.010 and done[1].start < done[0].finish
    assert done[0].slot != done[1].slot


def test_admission_respects_the_budget_and_rejects_oversized_jobs():
    clock = serve.VirtualClock()
    ex = _executor(clock)
    jobs = _jobs(rate=1000.0, count=30, footprint=300)
    jobs[7] = serve.Job(7, jobs[7].arrival, jobs[7].payload, footprint=5000)
    st = {}
    done = serve.serve(jobs, ex, clock, hbm_budget=1000, slots=8, stats=st)
    assert st["peak_reserved"] <= 1000 and st["peak_running"] == 3   # 3 x 300 <= 1000 < 4 x 300
    # never more than three running at any instant
    spans = [(d.start, d.finish) for d in done if d.error is None]
    for t in sorted(s for s, _ in spans):
        assert sum(1 for s, f in spans if s <= t < f) <= 3
    bad = [d for d in done if d.error]
    assert [d.jid for d in bad] == [7]
    assert sum(1 for d in done if d.error is None) == 29


def test_a_failing_job_fails_alone():
    clock = serve.VirtualClock()
    ex = _executor(clock, fail_ids=(5,))
    jobs = _jobs(rate=800.0, count=20)
    done = serve.serve(jobs, ex, clock, hbm_budget=10_000, slots=4)
    errs = {d.jid for d in done if d.error}
    assert errs == {5}
    assert len(done) == 20


def test_one_slot_is_fifo():
    clock = serve.VirtualClock()
    ex = _executor(clock)
    jobs = _jobs(rate=50.0, count=15)
    done = serve.serve(jobs, ex, clock, hbm_budget=10_000, slots=1)
    assert [jid for jid, _, _ in ex.submitted] == list(range(15))
    d = sorted(done, key=lambda x: x.start)
    assert all(a.finish <= b.start for a, b in zip(d, d[1:]))
    s = serve.summarize(done, clock.now())
    assert s["ok"] == 15 and s["p99_ms"] >= s["p50_ms"] > 0


def test_continuous_beats_fifo_under_load():
    """Above FIFO's capacity (one job per 10 ms, 150 jobs/s offered), slots
    sharing the device (each extra running job stretches a new one by 30%)
    still finish more jobs per second and with a lower p99."""
    jobs = _jobs(rate=150.0, count=80)
    res = {}
    for slots in (1, 4):
        clock = serve.VirtualClock()
        done = serve.serve(jobs, _executor(clock), clock, hbm_budget=100_000, slots=slots)
        res[slots] = serve.summarize(done, clock.now())
    assert res[4]["jobs_per_s"] > res[1]["jobs_per_s"]
    assert res[4]["p99_ms"] < res[1]["p99_ms"]


def test_work_budget_keeps_large_jobs_apart_but_lets_small_ones_run_beside():
    """Two large jobs (work 100) never overlap under a work budget of 125;
    small jobs (work 1) run beside a large one; a job above the budget runs
    once nothing else does."""
    clock = serve.VirtualClock()
    ex = _executor(clock, base_s=0.020, share=0.0)
    A = synth.random_a(np.random.default_rng(3), 10, 20, 0.2)
    jobs = [serve.Job(0, 0.000, A, 1, "large", 100), serve.Job(1, 0.001, A, 1, "large", 100),
            serve.Job(2, 0.002, A, 1, "small", 1), serve.Job(3, 0.003, A, 1, "small", 1),
            serve.Job(4, 0.004, A, 1, "huge", 500)]
    done = {d.jid: d for d in serve.serve(jobs, ex, clock, hbm_budget=100, slots=4, work_cap=125)}
    assert done[1].start >= done[0].finish                     # the two large ones one after the other
    assert done[2].start == 0.002 and done[2].start < done[0].finish   # small beside the first large
    assert done[3].start == 0.003
    others = [d for k, d in done.items() if k != 4]
    assert all(done[4].start >= d.finish for d in others)     # above the budget: alone
    assert all(d.error is None for d in done.values())


def test_summary_splits_latency_by_kind():
    d = [serve.Done(0, 0.0, 0.0, 0.1, 0, kind="large"), serve.Done(1, 0.0, 0.0, 0.01, 1, kind="tiny")]
    s = serve.summarize(d, 1.0)
    assert s["p50_ms_large"] > s["p50_ms_tiny"] > 0


def test_footprint_estimate_grows_with_size():
    small = serve.footprint_bytes(200, 5e4, 1.2e5, 1, 3e3)
    big = serve.footprint_bytes(3e4, 4e7, 1.5e8, 2, 1.6e6)
    assert 0 < small < big
