"""Batched and served forms on the GPU: every instance's result equals its
solo run (same kernels' arithmetic, exact merges: bitwise) and its oracle
run (parity rules of tests/parity.py)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2512_12094_amd import workloads as W
from tests.parity import compare_expectation, compare_terms

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_12094_amd import _lib
    _lib.lib()
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    return dict(torch=torch, stream=stream, handle=int(stream.cuda_stream),
                alloc=_lib.TorchAllocator(0))


def prefix(prog, k):
    return W.Program(prog.name + f"[:{k}]", prog.n, prog.group, prog.obs,
                     prog.sublayers[len(prog.sublayers) - k:], prog.bloch, dict(prog.meta))


def test_batch_config4_instances(gpu):
    """Instances of the batched ring workload (uneven n from 16 to 64, both
    merge key widths), two sub-layers each, in one batch."""
    from paper_2512_12094_amd import driver, _lib as L
    progs = [prefix(p, 2 + (k % 3)) for k, p in enumerate(W.config4()[:12])]
    print("[case] batch of", [(p.n, len(p.sublayers)) for p in progs], flush=True)
    for gps in (1, 4):
        L.pp_set_tuning(gates_per_step=gps)
        e, sets, dprogs, wall = driver.batch_propagate(progs, gpu["handle"], gpu["alloc"])
        for p, ei, s in zip(progs, e, sets):
            ref = O.run_program(p)
            compare_terms(s.as_dict(), ref.terms, p.meta["eps"], what=p.name)
            compare_expectation(ei, ref.expectation, ref.terms, what=p.name)
            assert s.counters() == (ref.propagated, ref.merged), p.name
            solo = driver.propagate_program(p, stream=gpu["handle"], allocator=gpu["alloc"])
            assert ei == solo.expectation, (p.name, ei, solo.expectation)
            s.close()
        for d in dprogs:
            d.close()
    L.pp_set_tuning(gates_per_step=4)


def test_batch_config4_instances_full_depth(gpu):
    """Twelve instances of the batched ring workload at their full depth
    (n = 16 to 64, 15 to 66 sub-layers, eps 2e-6 to 9e-5: the ones the
    oracle finishes in seconds), in one batch with layer ops: sets,
    coefficients, expectations and work counters against the oracle, and
    expectations bitwise equal to the solo runs."""
    from paper_2512_12094_amd import driver
    pick = (11, 19, 20, 22, 25, 27, 29, 32, 34, 44, 47, 54)
    allp = W.config4()
    progs = [allp[i] for i in pick]
    print("[case] full-depth batch", [(p.n, len(p.sublayers)) for p in progs], flush=True)
    e, sets, dprogs, wall = driver.batch_propagate(progs, gpu["handle"], gpu["alloc"])
    for p, ei, s in zip(progs, e, sets):
        ref = O.run_program(p)
        compare_terms(s.as_dict(), ref.terms, p.meta["eps"], what=p.name)
        compare_expectation(ei, ref.expectation, ref.terms, what=p.name)
        assert s.counters() == (ref.propagated, ref.merged), p.name
        solo = driver.propagate_program(p, stream=gpu["handle"], allocator=gpu["alloc"])
        assert ei == solo.expectation, (p.name, ei, solo.expectation)
        s.close()
    for d in dprogs:
        d.close()


def test_serve_alone_equals_in_the_mix(gpu):
    """Continuous batching: jobs arriving while others run; each result is
    the job's solo result (bitwise) and matches the oracle."""
    from paper_2512_12094_amd import driver, serve
    rng = np.random.default_rng(3)
    jobs = []
    t = 0.0
    for k in range(14):
        t += float(rng.exponential(0.002))
        if k % 3 == 2:
            n = int(rng.choice([6, 8, 10]))
            prog = W.heisenberg_all_to_all(n, int(rng.integers(1, 3)), 0.05, eps=1e-6,
                                           p=float(rng.uniform(0, 1e-2)), name=f"s{k}_n{n}")
        else:
            n = int(rng.choice([8, 12, 16, 20, 40]))
            prog = W.xxz_ring(n, int(rng.integers(1, 4)), float(rng.uniform(0.01, 0.1)),
                              float(rng.uniform(0.5, 2)), eps=float(10 ** rng.uniform(-6, -3)),
                              name=f"z{k}_n{n}")
        jobs.append(W.Job(t, prog))
    print("[case] serve", len(jobs), "jobs", flush=True)
    eng = serve.GpuEngine(gpu["handle"], gpu["alloc"], steps_per_iter=16)
    srv = serve.Server(eng, hbm_budget=5e9, max_active=6)
    res = srv.run(jobs)
    assert srv.peak_used <= 5e9
    for j, r in zip(jobs, res):
        solo = driver.propagate_program(j.program, stream=gpu["handle"], allocator=gpu["alloc"])
        assert r.expectation == solo.expectation, (r.name, r.expectation, solo.expectation)
        ref = O.run_program(j.program)
        compare_expectation(r.expectation, ref.expectation, ref.terms, what=r.name)
        assert r.units == ref.propagated + ref.merged, r.name
        assert r.finished >= r.arrival


def test_serve_config5_jobs_at_their_sizes(gpu):
    """Jobs of the served workload itself: five of its ring jobs at full
    depth (n = 16, 24) and its all-to-all S_n jobs at n = 32, 64 and 128
    over their first two sub-layers (their full depth passes the store limit
    the served leg uses), arriving together.  Each result equals the job's
    solo run bitwise and the oracle's by the FP64 rules, with equal work."""
    from paper_2512_12094_amd import driver, serve
    want_rings = {"c5_101_z16", "c5_109_z16", "c5_124_z16", "c5_151_z16", "c5_160_z24"}
    picked, sn_seen = [], set()
    for j in W.config5(count=200):
        p = j.program
        if p.name in want_rings:
            picked.append(W.Job(j.arrival * 1e-3, p))
        elif p.group == W.GROUP_SN and p.n in (32, 64, 128) and p.n not in sn_seen:
            sn_seen.add(p.n)
            picked.append(W.Job(j.arrival * 1e-3, prefix(p, 2)))
    assert len(picked) == 8, [j.program.name for j in picked]
    print("[case] serve config5 jobs", [(j.program.name, len(j.program.sublayers))
                                        for j in picked], flush=True)
    eng = serve.GpuEngine(gpu["handle"], gpu["alloc"], steps_per_iter=16)
    srv = serve.Server(eng, hbm_budget=20e9, max_active=8)
    res = srv.run(picked)
    for j, r in zip(picked, res):
        solo = driver.propagate_program(j.program, stream=gpu["handle"], allocator=gpu["alloc"])
        assert r.expectation == solo.expectation, (r.name, r.expectation, solo.expectation)
        ref = O.run_program(j.program)
        compare_expectation(r.expectation, ref.expectation, ref.terms, what=r.name)
        assert r.units == ref.propagated + ref.merged, r.name


def test_batch_instance_failure_is_isolated(gpu):
    """An instance that exceeds its store limit stops (-1); the others finish."""
    from paper_2512_12094_amd import driver, _lib as L
    print("[case] batch failure isolation", flush=True)
    good = W.xxz_ring(12, 2, 0.2, 1.0, eps=1e-6, name="good")
    bad = W.config1().with_group("none")
    sets = [driver.PauliSet.from_program(p, None, gpu["handle"], gpu["alloc"])
            for p in (good, bad)]
    L.pp_set_max_terms(sets[1].h, 5000)
    dps = [driver.device_program(p) for p in (good, bad)]
    done, e = L.pp_batch_step([s.h for s in sets], [d.h for d in dps], gpu["handle"], 100000)
    assert list(done) == [1, -1]
    ref = O.run_program(good)
    compare_expectation(e[0], ref.expectation, ref.terms, what="good")
    for s in sets:
        s.close()


def test_batch_promotes_a_large_instance(gpu):
    """A batch holding one instance that grows past 2^18 stored entries (the
    at-scale Z_32 ring over 12 sub-layers) beside small ones: the large one
    leaves the batch and finishes on the one-instance path (partitioned
    merges), the others stay batched.  Every instance equals its solo run
    bitwise (set, coefficients, expectation, counters); the small ones also
    match the oracle."""
    from paper_2512_12094_amd import driver, _lib as L
    big = W.xxz_ring(32, 5, 0.2, 1.5, eps=1e-6, wmax=12, obs=W.sum_ring_pairs(32, "X"),
                     name="ring32_scale")
    progs = [prefix(big, 12)] + [prefix(p, 2) for p in W.config4()[:5]]
    print("[case] batch with a large instance", [(p.n, len(p.sublayers)) for p in progs],
          flush=True)
    old = L.pp_get_tuning()
    L.pp_set_tuning(graph_steps=8)                 # step boundaries inside the program
    try:
        e, sets, dprogs, wall = driver.batch_propagate(progs, gpu["handle"], gpu["alloc"])
    finally:
        L.pp_set_tuning(graph_steps=old["graph_steps"])
    assert L.pp_peak_terms(sets[0].h) >= 1 << 18
    assert L.pp_merge_stats(sets[0].h)["partitioned_merges"] >= 1
    for k, (p, ei, s) in enumerate(zip(progs, e, sets)):
        got = s.as_dict()
        cnt = s.counters()
        solo_ps = driver.PauliSet.from_program(p, None, gpu["handle"], gpu["alloc"])
        dp = driver.device_program(p)
        es = float(L.pp_batch_run([solo_ps.h], [dp.h], gpu["handle"])[0])
        assert ei == es, (p.name, ei, es)
        assert got == solo_ps.as_dict(), p.name
        assert cnt == solo_ps.counters(), p.name
        solo_ps.close()
        dp.close()
        if k:
            ref = O.run_program(p)
            compare_terms(got, ref.terms, p.meta["eps"], what=p.name)
        s.close()
    for d in dprogs:
        d.close()
