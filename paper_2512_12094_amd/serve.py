"""Served form: continuous batching of propagation jobs on one GPU.

Jobs (a `workloads.Program` each, with an arrival time) enter a FIFO queue.
Every iteration of the event loop

1. moves the jobs that have arrived into the waiting queue;
2. admits waiting jobs in order while their estimated memory (estimated
   peak terms x bytes per stored term) fits the HBM budget and a batch slot
   is free: the job's handle is created (Algorithm 1 step 1 on the device)
   and its program uploaded; its Pauli set then stays on the device;
3. advances every admitted job together by a few batched steps
   (pp_batch_step: one persistent launch per kernel kind serves all jobs);
4. retires finished jobs (expectation, latency = finish - arrival) and frees
   their memory; the estimator learns the job's peak store size as the
   device tracked it (pp_peak_terms); a job whose store outgrew its estimate
   is re-queued with four times the estimate (it restarts from its
   observable, nothing is reused), and rejected once it has failed at the
   largest estimate the store limit or the whole budget allows (its result
   then says so).  A failure also raises the starting estimate of later
   jobs of the same class.

Memory is accounted by the bytes the library would allocate for the job's
store at its limit (pp_store_bytes), and an estimate is lowered to what the
whole budget holds, so a job alone never exceeds it either.

Jobs that arrive while others run join at the next iteration.  The GPU work
goes through an engine object so the policy can be exercised on the CPU with
a fake engine (tests/test_serve.py).
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from .workloads import Program, n_words

# bytes of device memory per unit of store capacity (both halves of x, z, c,
# four alive arrays, gate table, merge table with 3-limb sums, partials)
_BYTES_PER_SLOT = {1: 2 * (8 + 8 + 8) + 4 + 2 * 8 + 2 * (8 + 24) + 1,
                   2: 2 * (16 + 16 + 8) + 4 + 2 * 8 + 2 * (8 + 24 + 4) + 4 * 8 + 4 + 1}


def bytes_per_term(n: int) -> int:
    """Device bytes per stored term, with the store's 4x growth headroom."""
    return 4 * _BYTES_PER_SLOT[min(2, n_words(n))]


@dataclass
class JobResult:
    name: str
    arrival: float
    admitted: float = math.nan
    finished: float = math.nan
    expectation: float = math.nan
    units: int = 0                # propagated + merged terms
    retries: int = 0
    est_terms: int = 0
    rejected: bool = False
    unfinished: bool = False      # stopped by the server's time budget

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Estimator:
    """Peak stored terms of a job, by class (group, n, eps decade), learned
    from finished jobs (largest seen x 2), with a prior for unseen classes;
    never above the store limit `cap_terms`."""

    def __init__(self, prior: int = 1 << 16, cap_terms: int = 1 << 28):
        self.prior, self.cap_terms = prior, cap_terms
        self.seen: dict = {}
        self.hopeless: set = set()   # classes that failed at the largest estimate

    @staticmethod
    def key(prog: Program):
        eps = prog.meta.get("eps", 0.0) or 1e-16
        return (prog.group, prog.n, int(math.floor(math.log10(eps))))

    def estimate(self, prog: Program) -> int:
        v = self.seen.get(self.key(prog))
        return min(self.cap_terms, 2 * v if v else self.prior)

    def observe(self, prog: Program, peak_terms: int):
        k = self.key(prog)
        self.seen[k] = max(self.seen.get(k, 0), int(peak_terms))

    def failed(self, prog: Program, store_terms: int):
        """A job of this class outgrew a store of `store_terms` entries: jobs
        of the class start from twice that (capped) from now on."""
        self.observe(prog, store_terms)

    def give_up(self, prog: Program):
        """A job of this class failed at the largest estimate allowed: later
        jobs of the class are rejected without running."""
        self.hopeless.add(self.key(prog))

    def is_hopeless(self, prog: Program) -> bool:
        return self.key(prog) in self.hopeless


class GpuEngine:
    """The device side: one handle and one uploaded program per job."""

    def __init__(self, stream: int, allocator=None, steps_per_iter: int = 32):
        from . import _lib as L
        from . import driver
        self.L, self.driver = L, driver
        self.stream, self.allocator = stream, allocator
        self.steps_per_iter = steps_per_iter

    def start(self, job_prog: Program, max_terms: int):
        ps = self.driver.PauliSet.from_program(job_prog, None, self.stream, self.allocator)
        self.L.pp_set_max_terms(ps.h, max_terms)
        dp = self.driver.device_program(job_prog)
        return (ps, dp)

    def step(self, handles):
        done, e = self.L.pp_batch_step([h[0].h for h in handles], [h[1].h for h in handles],
                                       self.stream, self.steps_per_iter)
        return done, e

    def finish(self, handle):
        """Work units and the largest store (entries) the job needed, as the
        device tracked it."""
        ps, _ = handle
        wc = self.L.pp_work_counters(ps.h)
        units = wc["propagated"] + wc["merged"]
        peak = max(self.L.pp_peak_terms(ps.h), 1)
        ps.close()
        return units, peak

    def job_bytes(self, prog: Program, est: int) -> int:
        """Device bytes of a job allowed `est` terms: its store at the limit
        it is started with (4 est entries), plus half that for the copy while
        the store last grew."""
        cap = max(4096, 4 * int(est))
        b = self.L.pp_store_bytes(prog.n, prog.group, cap)
        return b + b // 2

    def abort(self, handle):
        handle[0].close()


@dataclass
class Server:
    engine: object
    hbm_budget: float                      # bytes available to job stores
    max_active: int = 256
    estimator: Estimator = field(default_factory=Estimator)
    clock: object = time.perf_counter
    sleep: object = time.sleep
    max_retries: int = 8
    growth: int = 4                        # estimate factor after a failure
    give_up_classes: bool = False          # reject later jobs of a class that failed
                                           # at the largest estimate, without running

    def job_bytes(self, prog: Program, est: int) -> float:
        fn = getattr(self.engine, "job_bytes", None)
        return fn(prog, est) if fn else est * bytes_per_term(prog.n)

    def fit_estimate(self, prog: Program, est: int) -> int:
        """The estimate, lowered if needed until the job fits the whole
        budget (a job alone may use all of it); 0 if not even the smallest
        store fits."""
        est = max(1, int(est))
        while est > 1024 and self.job_bytes(prog, est) > self.hbm_budget:
            est //= 2
        return est if self.job_bytes(prog, est) <= self.hbm_budget else 0

    def run(self, jobs, on_event=None, time_budget=None):
        """Serves `jobs` (objects with .arrival and .program); returns
        JobResult per job in input order.  With `time_budget` (seconds),
        jobs not finished by then are stopped and marked unfinished."""
        order = sorted(range(len(jobs)), key=lambda i: jobs[i].arrival)
        pending = deque(order)
        waiting = deque()
        active = []                       # (index, handle, bytes, est)
        results = [JobResult(getattr(j.program, "name", str(i)), j.arrival)
                   for i, j in enumerate(jobs)]
        used = 0.0
        self.peak_used = 0.0
        t0 = self.clock()
        while pending or waiting or active:
            now = self.clock() - t0
            if time_budget is not None and now > time_budget:
                for i, handle, need, est in active:
                    self.engine.abort(handle)
                    results[i].unfinished = True
                for i in list(waiting) + list(pending):
                    results[i].unfinished = True
                break
            while pending and jobs[pending[0]].arrival <= now:
                waiting.append(pending.popleft())
            # admission, in arrival order
            while waiting and len(active) < self.max_active:
                i = waiting[0]
                prog = jobs[i].program
                est = self.fit_estimate(prog, max(results[i].est_terms,
                                                  self.estimator.estimate(prog)))
                if est == 0 or (self.give_up_classes and self.estimator.is_hopeless(prog)):
                    waiting.popleft()
                    results[i].rejected, results[i].finished = True, now
                    if on_event:
                        on_event("reject", i, used)
                    continue
                need = self.job_bytes(prog, est)
                if used + need > self.hbm_budget:
                    break
                waiting.popleft()
                results[i].est_terms = est
                results[i].admitted = self.clock() - t0
                handle = self.engine.start(prog, 4 * est)
                active.append((i, handle, need, est))
                used += need
                self.peak_used = max(self.peak_used, used)
                if on_event:
                    on_event("admit", i, used)
            if not active:
                if pending:
                    self.sleep(max(0.0, jobs[pending[0]].arrival - (self.clock() - t0)))
                continue
            done, e = self.engine.step([a[1] for a in active])
            now = self.clock() - t0
            keep = []
            for (i, handle, need, est), dn, ei in zip(active, done, e):
                if dn == 1:
                    units, peak = self.engine.finish(handle)
                    r = results[i]
                    r.finished, r.expectation, r.units = now, float(ei), units
                    self.estimator.observe(jobs[i].program, peak)
                    used -= need
                    if on_event:
                        on_event("finish", i, used)
                elif dn < 0:              # outgrew its estimate: restart, larger
                    self.engine.abort(handle)
                    used -= need
                    r = results[i]
                    r.retries += 1
                    new_est = self.growth * est
                    prog = jobs[i].program
                    self.estimator.failed(prog, 4 * est)
                    if (r.retries > self.max_retries or est >= self.estimator.cap_terms or
                            self.fit_estimate(prog, min(new_est, self.estimator.cap_terms))
                            <= est):
                        r.rejected, r.finished = True, now
                        self.estimator.give_up(prog)
                        if on_event:
                            on_event("reject", i, used)
                    else:                 # the last try is at the limit itself
                        r.est_terms = min(new_est, self.estimator.cap_terms)
                        waiting.appendleft(i)
                        if on_event:
                            on_event("requeue", i, used)
                else:
                    keep.append((i, handle, need, est))
            active = keep
        return results


def summarize(results, wall: float) -> dict:
    """Latency percentiles over the completed jobs, throughput over all
    completed work, counts of retries, rejections and unfinished jobs."""
    done = [r for r in results if not r.rejected and not r.unfinished]
    lat = np.array([r.latency for r in done]) if done else np.array([math.nan])
    units = sum(r.units for r in done)
    return dict(jobs=len(results), completed=len(done),
                rejected=sum(r.rejected for r in results),
                unfinished=sum(r.unfinished for r in results),
                p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                mean_s=float(lat.mean()),
                terms_per_s=units / wall if wall > 0 else float("nan"), wall_s=wall,
                retries=int(sum(r.retries for r in results)))
