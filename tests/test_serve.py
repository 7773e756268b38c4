"""Serving policy on the CPU with a fake engine and a fake clock: admission
never exceeds the memory budget, jobs that arrive later join while others
run, a job that outgrows its estimate is re-queued with a doubled estimate,
latency is finish - arrival."""
from dataclasses import dataclass

from paper_2512_12094_amd import serve, workloads as W


@dataclass
class FakeJob:
    arrival: float
    program: object


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-3)


class FakeEngine:
    """A job needs `work` steps; it fails (outgrows its store) when its true
    peak exceeds the store limit it was started with."""

    def __init__(self, clock, work, peak, step_time=0.01):
        self.clock, self.work, self.peak, self.step_time = clock, work, peak, step_time
        self.started = []

    def start(self, prog, max_terms):
        h = dict(name=prog.name, left=self.work[prog.name], max_terms=max_terms)
        self.started.append((prog.name, max_terms))
        return h

    def step(self, handles):
        self.clock.t += self.step_time
        done, e = [], []
        for h in handles:
            if self.peak[h["name"]] > h["max_terms"]:
                done.append(-1)
            else:
                h["left"] -= 1
                done.append(1 if h["left"] <= 0 else 0)
            e.append(float(len(h["name"])))
        return done, e

    def finish(self, h):
        return 100, self.peak[h["name"]]

    def abort(self, h):
        pass


def make_jobs(k, gap=0.005):
    jobs = []
    for i in range(k):
        p = W.xxz_ring(16, 1, 0.1, 1.0, eps=1e-4, name=f"j{i}")
        jobs.append(FakeJob(i * gap, p))
    return jobs


def test_budget_is_never_exceeded_and_jobs_overlap():
    clock = FakeClock()
    jobs = make_jobs(20)
    eng = FakeEngine(clock, {j.program.name: 5 for j in jobs},
                     {j.program.name: 1000 for j in jobs})
    budget = 3.5 * (1 << 16) * serve.bytes_per_term(16)   # room for 3 jobs
    events = []
    srv = serve.Server(eng, budget, clock=clock, sleep=clock.sleep)
    res = srv.run(jobs, on_event=lambda kind, i, used: events.append((kind, i, used)))
    assert all(r.finished >= r.arrival for r in res)
    assert srv.peak_used <= budget
    # continuous batching: a job admitted while another was active
    active, overlapped = set(), False
    for kind, i, used in events:
        if kind == "admit":
            overlapped |= bool(active)
            active.add(i)
        elif kind == "finish":
            active.discard(i)
    assert overlapped
    # FIFO admission
    admits = [i for kind, i, _ in events if kind == "admit"]
    assert admits == sorted(admits)


def test_underestimate_is_requeued_with_larger_estimate():
    clock = FakeClock()
    jobs = make_jobs(3)
    big = jobs[1].program.name
    peak = {j.program.name: 10 for j in jobs}
    peak[big] = 12 * (1 << 16)             # beyond the prior's store limit
    eng = FakeEngine(clock, {j.program.name: 3 for j in jobs}, peak)
    srv = serve.Server(eng, 1e15, clock=clock, sleep=clock.sleep)
    res = srv.run(jobs)
    assert res[1].retries == 1 and not res[1].rejected
    starts = [m for name, m in eng.started if name == big]
    # the failure at 4 x 2^16 raises the class estimate to twice that
    assert starts == [4 * (1 << 16), 32 * (1 << 16)]
    assert all(r.finished > 0 for r in res)


def test_job_beyond_the_store_limit_is_rejected_not_fatal():
    clock = FakeClock()
    jobs = make_jobs(3)
    jobs[0] = FakeJob(0.0, W.xxz_ring(24, 1, 0.1, 1.0, eps=1e-4, name="huge"))
    huge = "huge"
    peak = {j.program.name: 10 for j in jobs}
    peak[huge] = 1 << 40
    eng = FakeEngine(clock, {j.program.name: 3 for j in jobs}, peak)
    srv = serve.Server(eng, 1e15, estimator=serve.Estimator(cap_terms=1 << 22), clock=clock,
                       sleep=clock.sleep)
    res = srv.run(jobs)
    assert res[0].rejected and not res[1].rejected and not res[2].rejected
    s = serve.summarize(res, 1.0)
    assert s["rejected"] == 1 and s["completed"] == 2
    # the huge job's last try was at the limit (4 x cap_terms entries)
    assert eng.started[-1][1] == 4 * (1 << 22) or ("huge", 4 * (1 << 22)) in eng.started
    # a later job of the class that outgrew the limit starts at the limit
    late = FakeJob(0.0, W.xxz_ring(24, 1, 0.1, 1.0, eps=1e-4, name="late"))
    eng.work["late"], eng.peak["late"] = 3, 10
    res2 = srv.run([late])
    assert not res2[0].rejected and eng.started[-1] == ("late", 4 * (1 << 22))


def test_estimator_learns_from_finished_jobs():
    est = serve.Estimator(prior=100)
    p = W.xxz_ring(16, 1, 0.1, 1.0, eps=1e-4)
    assert est.estimate(p) == 100
    est.observe(p, 700)
    assert est.estimate(p) == 1400


def test_summary():
    rs = [serve.JobResult("a", 0.0, finished=1.0, units=10),
          serve.JobResult("b", 0.5, finished=3.5, units=30)]
    s = serve.summarize(rs, 4.0)
    assert s["terms_per_s"] == 10.0 and s["jobs"] == 2
    assert 1.0 <= s["p50_s"] <= 3.0


def test_a_job_alone_never_exceeds_the_budget():
    """An estimate larger than the whole budget is lowered to what the budget
    holds (the job then runs alone within it); a job whose smallest store
    does not fit is rejected without running."""
    clock = FakeClock()
    jobs = make_jobs(3)
    eng = FakeEngine(clock, {j.program.name: 3 for j in jobs},
                     {j.program.name: 500 for j in jobs})
    per_term = serve.bytes_per_term(16)
    budget = 4000 * per_term
    est = serve.Estimator(prior=1 << 20)                 # far above the budget
    srv = serve.Server(eng, budget, estimator=est, clock=clock, sleep=clock.sleep)
    res = srv.run(jobs)
    assert srv.peak_used <= budget
    assert all(not r.rejected for r in res)
    assert all(max_terms <= 4 * 4000 for _, max_terms in eng.started)
    tiny = serve.Server(FakeEngine(clock, {j.program.name: 1 for j in jobs},
                                   {j.program.name: 1 for j in jobs}),
                        10 * per_term, clock=clock, sleep=clock.sleep)
    assert all(r.rejected for r in tiny.run(jobs))


def test_time_budget_stops_unfinished_jobs():
    clock = FakeClock()
    jobs = make_jobs(10, gap=0.0)
    eng = FakeEngine(clock, {j.program.name: 1000 for j in jobs},
                     {j.program.name: 10 for j in jobs})
    srv = serve.Server(eng, 1e12, clock=clock, sleep=clock.sleep)
    res = srv.run(jobs, time_budget=0.5)
    assert all(r.unfinished for r in res)
    s = serve.summarize(res, 0.5)
    assert s["completed"] == 0 and s["unfinished"] == 10


def test_estimator_learns_the_peak_the_engine_reports():
    clock = FakeClock()
    jobs = make_jobs(2)
    eng = FakeEngine(clock, {j.program.name: 2 for j in jobs},
                     {j.program.name: 777 for j in jobs})
    est = serve.Estimator(prior=1 << 12)
    serve.Server(eng, 1e12, estimator=est, clock=clock, sleep=clock.sleep).run(jobs)
    assert est.estimate(jobs[0].program) == 2 * 777


def test_give_up_on_a_class_that_failed_at_the_limit():
    """With give_up_classes, a later job of a class that failed at the
    largest estimate is rejected without being started."""
    clock = FakeClock()
    jobs = [FakeJob(5.0 * i, W.xxz_ring(24, 1, 0.1, 1.0, eps=1e-4, name=f"h{i}")) for i in range(3)]
    eng = FakeEngine(clock, {j.program.name: 3 for j in jobs},
                     {j.program.name: 1 << 40 for j in jobs})
    srv = serve.Server(eng, 1e15, estimator=serve.Estimator(cap_terms=1 << 20), clock=clock,
                       sleep=clock.sleep, give_up_classes=True)
    res = srv.run(jobs)
    assert all(r.rejected for r in res)
    started = {name for name, _ in eng.started}
    assert started == {"h0"}
