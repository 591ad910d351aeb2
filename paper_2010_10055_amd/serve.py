"""Serving loop for layout jobs: overlap, overlap graph, reduction, on one GPU.

A job is one read set: C = A A^T, the overlap graph R built on the device
from C's seeds (dibella_r_from_seeds: suffix and orientation from the first
stored seed; the second seed's agreement and the density of shared k-mers
along the overlap stand in for the alignment that prunes C in the paper's
pipeline), then S = TR(R).  C, R and S stay on the device between the stages.

Scheduling is continuous batching over `slots` execution slots.  Each slot
is a host thread with its own HIP stream, so the work of admitted jobs
overlaps on the device (the library is thread-safe per stream).  Jobs arrive
over time (Poisson) and wait in a queue; whenever a slot is idle, the first
waiting job (in arrival order) whose estimated footprint (A, its transpose
and sort buffers, C, R and scratch) fits the HBM budget still unreserved is
admitted on it, if its estimated work (semiring products) also fits the work
budget beside the jobs already running.  The HBM budget is the measured free
device memory at the start of the run (or less, if the caller says so).  The
work budget keeps jobs that each fill the GPU from running side by side,
where they only slow each other down, while small jobs still run beside
them.  A job whose footprint exceeds the whole HBM budget fails alone; a job
above the work budget runs when nothing else does.  A job that arrives while others run starts as
soon as a slot and memory allow, not when the running ones have finished.
One slot is the FIFO baseline (a queue alone, one job on the device at a
time), on the same scheduler and trace.

The scheduler needs an executor (submit a job to a slot; wait for finished
jobs) and a clock, so it is tested on the CPU with a virtual-time executor
and a virtual clock.
"""
from __future__ import annotations

import dataclasses
import math
import queue as _queue
import threading
import time
from typing import Callable, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Job:
    jid: int
    arrival: float          # seconds from the start of the run
    payload: object         # executor-specific inputs
    footprint: int          # estimated device bytes while running
    kind: str = "job"
    work: int = 0           # estimated device work (semiring products)


@dataclasses.dataclass
class Done:
    jid: int
    arrival: float
    start: float
    finish: float
    slot: int
    result: object = None
    error: Optional[str] = None
    kind: str = "job"

    @property
    def latency(self) -> float:
        return self.finish - self.arrival


def poisson_arrivals(rng: np.random.Generator, count: int, rate: float) -> np.ndarray:
    """Arrival times of a Poisson process of `rate` jobs/s."""
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def footprint_bytes(nrows: int, nnz_a: int, products: int, min_shared: int, nnz_r_est: int) -> int:
    """Estimated device bytes of one job while it runs: A (12 B/entry) and its
    sort pairs, segments and transpose (32 B/entry), per-row arrays
    (~200 B/row), the output-column scratch and C (4 + 24 B per possible
    output entry, at most products / min_shared), and R with its reduction
    buffers (~30 B/entry)."""
    out = products // max(1, min_shared)
    return int(44 * nnz_a + 200 * nrows + 28 * out + 30 * nnz_r_est)


class WallClock:
    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def wait_until(self, t: float) -> None:
        d = t - self.now()
        if d > 0:
            time.sleep(d)


class VirtualClock:
    """A clock that only moves when told (for tests)."""

    def __init__(self):
        self.t = 0.0

    def now(self) -> float:
        return self.t

    def wait_until(self, t: float) -> None:
        self.t = max(self.t, t)

    def advance(self, dt: float) -> None:
        self.t += dt


def serve(jobs: Sequence[Job], executor, clock, hbm_budget: int, slots: int = 4,
          stats: Optional[dict] = None, on_done: Optional[Callable[[Done], None]] = None,
          work_cap: Optional[int] = None) -> List[Done]:
    """Run `jobs` through continuous admission over `slots` slots (work_cap:
    the most estimated work running at once; None = no limit).

    executor.submit(job, slot) starts a job; executor.wait(timeout) blocks
    until at least one job has finished or `timeout` seconds have passed
    (None: until a job finishes) and returns [(jid, result, error, finish)]
    for the finished ones.  `stats`, if given, receives the peak reserved
    footprint and the peak number of jobs running at once; `on_done` is
    called with every finished job."""
    order = sorted(jobs, key=lambda j: j.arrival)
    waiting: List[Job] = []
    done: List[Done] = []
    idle = list(range(slots))
    running = {}   # jid -> (job, slot, start)
    reserved = working = 0
    peak_reserved = peak_running = 0
    nxt = 0
    while nxt < len(order) or waiting or running:
        now = clock.now()
        while nxt < len(order) and order[nxt].arrival <= now:
            waiting.append(order[nxt])
            nxt += 1
        # admission in arrival order: the first waiting jobs that fit a slot
        # and the unreserved budget start now
        rest: List[Job] = []
        for j in waiting:
            if j.footprint > hbm_budget:
                done.append(Done(j.jid, j.arrival, now, now, -1, None, "footprint exceeds the HBM budget", j.kind))
            elif (idle and reserved + j.footprint <= hbm_budget and
                  (work_cap is None or not running or working + j.work <= work_cap)):
                slot = idle.pop(0)
                reserved += j.footprint
                working += j.work
                running[j.jid] = (j, slot, now)
                executor.submit(j, slot)
            else:
                rest.append(j)
        waiting = rest
        peak_reserved = max(peak_reserved, reserved)
        peak_running = max(peak_running, len(running))
        timeout = max(0.0, order[nxt].arrival - now) if nxt < len(order) else None
        if running:
            for jid, result, error, finish in executor.wait(timeout):
                j, slot, start = running.pop(jid)
                reserved -= j.footprint
                working -= j.work
                idle.append(slot)
                done.append(Done(jid, j.arrival, start, finish, slot, result, error, j.kind))
                if on_done:
                    on_done(done[-1])
        elif timeout is not None:
            clock.wait_until(order[nxt].arrival)
        else:   # nothing runs and nothing arrives: every waiting job was admitted or failed
            assert not waiting
    if stats is not None:
        stats.update(peak_reserved=peak_reserved, peak_running=peak_running)
    return done


def summarize(done: Sequence[Done], wall: float) -> dict:
    ok = [d for d in done if d.error is None]
    lat = np.array([d.latency for d in ok]) if ok else np.zeros(1)
    out = {"jobs": len(done), "ok": len(ok), "failed": len(done) - len(ok),
           "jobs_per_s": len(ok) / wall if wall > 0 else float("inf"),
           "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
           "mean_ms": float(lat.mean() * 1e3), "wall_s": wall}
    kinds = sorted({d.kind for d in ok})
    if len(kinds) > 1:
        for k in kinds:
            lk = np.array([d.latency for d in ok if d.kind == k])
            out[f"p50_ms_{k}"] = float(np.percentile(lk, 50) * 1e3)
            out[f"p99_ms_{k}"] = float(np.percentile(lk, 99) * 1e3)
    return out


class VirtualExecutor:
    """Executor on a virtual clock (for the scheduler's CPU tests): a job
    runs `run(payload)` at once and finishes `duration(job, running)` seconds
    after its start, `running` being the number of jobs already running when
    it starts; a job whose id is in `fail_ids` raises."""

    def __init__(self, clock: VirtualClock, run: Callable, duration: Callable, fail_ids=()):
        self.clock, self.run, self.duration, self.fail_ids = clock, run, duration, set(fail_ids)
        self.pending = []   # (finish, seq, jid, result, error)
        self.submitted = []  # (jid, slot, start)
        self.seq = 0

    def submit(self, job: Job, slot: int) -> None:
        t = self.clock.now()
        self.submitted.append((job.jid, slot, t))
        try:
            if job.jid in self.fail_ids:
                raise RuntimeError("bad job")
            res, err = self.run(job.payload), None
        except Exception as ex:
            res, err = None, f"{type(ex).__name__}: {ex}"
        self.pending.append((t + self.duration(job, len(self.pending)), self.seq, job.jid, res, err))
        self.seq += 1

    def wait(self, timeout):
        if not self.pending:
            return []
        first = min(self.pending)
        deadline = math.inf if timeout is None else self.clock.now() + timeout
        if first[0] > deadline:
            self.clock.wait_until(deadline)
            return []
        self.clock.wait_until(first[0])
        out = [p for p in self.pending if p[0] <= self.clock.now()]
        self.pending = [p for p in self.pending if p[0] > self.clock.now()]
        return [(jid, res, err, fin) for fin, _, jid, res, err in sorted(out)]


# ---------------------------------------------------------------------------
# GPU side
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class LayoutInputs:
    """Device-resident inputs of one layout job (A with strand bits in its
    values, read lengths) and its parameters; host copies for checking."""
    A: object                # CSRTensors, values (position << 1) | strand
    read_len: object         # int32 device tensor
    k: int
    min_shared: int
    min_overlap: int
    max_drift: int
    min_density: int
    fuzz: int
    host_A: object = None    # synth.CSR (for the oracle in tests)
    host_len: object = None  # numpy int32


def density_threshold(error_rate: float, k: int, fraction: float = 0.4) -> int:
    """Shared k-mers per 10 kbp a pair must reach: `fraction` of the rate at
    which two reads with independent errors at `error_rate` share the k-mers
    of a true overlap (a k-mer is shared where both reads hold it without
    error: (1 - e)^(2k) per position)."""
    return max(1, int(round(fraction * 10000 * (1.0 - error_rate) ** (2 * k))))


def run_layout(inp: LayoutInputs):
    """One job on the current stream: C = A A^T, R from C's seeds, S = TR(R).
    Returns (C, R, S, passes); everything stays on the device."""
    import paper_2010_10055_amd as db
    C = db.overlap(inp.A, inp.min_shared)
    R = db.r_from_seeds(C, inp.read_len, inp.k, inp.min_overlap, inp.max_drift, inp.min_density)
    S, it = db.transitive_reduce(R, inp.fuzz)
    return C, R, S, it


def hbm_free_bytes(device: str = "cuda:0") -> int:
    """Device memory a run can still use: free memory plus what PyTorch's
    caching allocator holds without using."""
    import torch
    free, _ = torch.cuda.mem_get_info(device)
    return int(free + torch.cuda.memory_reserved(device) - torch.cuda.memory_allocated(device))


class GpuSlots:
    """Executor with one host thread and one HIP stream (default priority)
    per slot.  A worker runs its job on its stream, waits for that stream
    only, and reports the finish time; results are kept only if asked
    (config-3-sized results are gigabytes each)."""

    def __init__(self, slots: int, clock, run: Callable = run_layout, keep_results: bool = False,
                 device: str = "cuda:0"):
        import torch
        self.clock, self.run, self.keep, self.device = clock, run, keep_results, torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        self.inbox = [_queue.Queue() for _ in range(slots)]
        self.finished = _queue.Queue()
        self.threads = [threading.Thread(target=self._worker, args=(k,), daemon=True) for k in range(slots)]
        for t in self.threads:
            t.start()

    def _worker(self, k: int) -> None:
        import torch
        s = self.streams[k]
        while True:
            job = self.inbox[k].get()
            if job is None:
                return
            res = err = None
            try:
                with torch.cuda.device(self.device), torch.cuda.stream(s):
                    res = self.run(job.payload)
                s.synchronize()
            except Exception as ex:
                err = f"{type(ex).__name__}: {ex}"
                try:
                    s.synchronize()
                except Exception:
                    pass
            fin = self.clock.now()
            self.finished.put((job.jid, res if self.keep else None, err, fin))

    def submit(self, job: Job, slot: int) -> None:
        self.inbox[slot].put(job)

    def wait(self, timeout):
        try:
            out = [self.finished.get(timeout=timeout)]
        except _queue.Empty:
            return []
        while True:
            try:
                out.append(self.finished.get_nowait())
            except _queue.Empty:
                return out

    def close(self) -> None:
        for q in self.inbox:
            q.put(None)
        for t in self.threads:
            t.join()


def pool_entry(w, device: str = "cuda:0", min_overlap=None, max_drift: int = 150, keep_host: bool = False):
    """One device-resident job input from a generated workload whose A
    carries strand bits in its values: (name, LayoutInputs, footprint,
    products)."""
    import torch
    import paper_2010_10055_amd as db
    from . import synth
    lens = np.diff(w.reads.offsets).astype(np.int32)
    mo = (1 if w.name == "tiny" else 1000) if min_overlap is None else min_overlap
    inp = LayoutInputs(db.CSRTensors.from_numpy(w.A, device), torch.as_tensor(lens, device=device),
                       w.k, w.min_shared, mo, max_drift, density_threshold(w.error_rate, w.k), w.fuzz,
                       w.A if keep_host else None, lens if keep_host else None)
    products = synth.overlap_products(w.A)
    fp = footprint_bytes(w.A.nrows, w.A.nnz, products, w.min_shared, 80 * w.A.nrows)
    return (w.name, inp, fp, products)


def make_pool(kinds: Sequence[tuple], device: str = "cuda:0", min_overlap=None, max_drift: int = 150,
              keep_host: bool = False, log=lambda s: None):
    """Pre-generated device-resident instances: kinds = [(name, count,
    seed0, scale)] with workload names of the generator, built with strand
    bits in A's values.  Returns [(name, LayoutInputs, footprint, products)]."""
    from . import synth
    pool = []
    for name, count, seed0, scale in kinds:
        for q in range(count):
            w = synth.make_workload(name, seed=seed0 + q, device=device, scale=scale, strand_bit=True)
            pool.append(pool_entry(w, device, min_overlap, max_drift, keep_host))
            log(f"  pool {name}#{q}: reads {w.A.nrows}, nnz(A) {w.A.nnz}, footprint {pool[-1][2] / 2**30:.2f} GiB")
            del w
    return pool


def draw_jobs(rng: np.random.Generator, pool, count: int, rate: float, small_fraction: float = 0.1,
              small_kind: str = "tiny") -> List[Job]:
    """`count` jobs with Poisson arrivals; each job picks a pool instance:
    a `small_kind` one with probability small_fraction, else a large one."""
    small = [p for p in pool if p[0] == small_kind]
    large = [p for p in pool if p[0] != small_kind]
    times = poisson_arrivals(rng, count, rate)
    jobs = []
    for q in range(count):
        src = small if (small and (not large or rng.random() < small_fraction)) else large
        name, inp, fp, work = src[int(rng.integers(0, len(src)))]
        jobs.append(Job(q, float(times[q]), inp, fp, name, work))
    return jobs
