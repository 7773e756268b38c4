"""Throughput of symmetry-merging Pauli propagation on one MI355X.

One step = Algorithm 1 over the Z_32 XXZ ring workload (20 Trotter steps of
RXX(0.05), RYY(0.05), RZZ(0.075) sub-layers on all 32 bonds, O = sum X_i
X_{i+1}, eps = 1e-4, weight <= 8, symmetric product state): create + merge
the observable, 60 x (32 gates with exact merge and truncation, symmetry
merge, truncation), expectation.  Every step runs in the HIP kernels of
libpp.so through its C ABI on one stream; the inputs (gate tables) are
uploaded once per call, the term sets never leave the device.

value = (propagated + merged) terms / second, the paper's two work units
(Prop. 1: terms tested against a gate; records entering a merge), counted on
the device and equal to the oracle's counts (tests/test_gpu_parity.py).

The JSON line also carries: the same circuit without symmetry merging
(plain PP) and merged under the dihedral group D_n, the roofline of the dominant kernel (per-kernel durations from
HIP events recorded on the library's stream over the timed steps; HBM
traffic from the committed rocprofv3 counter summary when it matches the
current kernel sources), the exact-merge pass on a large record stream, the
batched form against a per-instance loop on a sample of the batched ring
workload, the served form (continuous batching, p50/p99 latency) on a
sample of the mixed job stream, and the CPU oracle timed on a bounded
prefix of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, bytes/s * 1e-9

METRIC = "Pauli terms propagated+merged/sec (sym PP vs plain PP); p50/p99 job latency"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-merge-pass", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-dihedral", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--event-every", type=int, default=4,
                    help="time every N-th run of back-to-back launches of one kernel "
                         "kind with HIP events")
    ap.add_argument("--merge-log2n", type=int, default=24)
    ap.add_argument("--merge-more", type=int, nargs="*", default=[26],
                    help="more merge-pass sizes (log2 of the records), 32 rotations each")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size (for PMC scaling)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-scale", action="store_true", help="skip the gate-at-scale leg")
    ap.add_argument("--no-ising", action="store_true", help="skip the Ising layers leg")
    ap.add_argument("--no-ising-family", action="store_true",
                    help="skip the Ising n = 3..20 family leg")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--batch-cap-terms", type=int, default=1 << 26,
                    help="store limit (entries) of a batched instance at full depth")
    ap.add_argument("--serve-count", type=int, default=600)
    ap.add_argument("--serve-seconds", type=float, default=30.0)
    ap.add_argument("--serve-cap-terms", type=int, default=1 << 25,
                    help="largest estimate a served job may reach (store = 4x)")
    ap.add_argument("--no-c3", action="store_true", help="skip the all-to-all leg")
    ap.add_argument("--cpu-pool-seconds", type=float, default=15.0)
    return ap.parse_args()


def gate_bytes(wc, W=1):
    """Algorithmic bytes of the apply step, priced per term-gate (Prop. 1's
    propagation unit): every live term tested against a rotation has its key
    read (16W B); every anticommuting one has its coefficient read and
    written (16 B); every appended child is written (16W + 8 B)."""
    return (16 * W * wc["propagated"] + 16 * wc["anticommuting"] +
            (16 * W + 8) * wc["appended"])


def gate_bytes_launch(wc, W=1):
    """The same bytes as a fused launch moves them: each key read once per
    launch (one launch applies up to three commuting rotations), each
    touched coefficient read and written once per launch."""
    return (16 * W * wc["gate_key_reads"] + 16 * wc["gate_coef_rw"] +
            (16 * W + 8) * wc["appended"])


def merge_bytes(wc, W=1):
    """Algorithmic bytes of a symmetry merge: every record read (16W + 8 B),
    every representative written (16W + 8 B)."""
    return (16 * W + 8) * (wc["merge_in"] + wc["merge_out"])


def run_steps(prog, group, steps, stream, alloc, profile, mode="program", layer_ops=1):
    """`steps` propagations; mode "program" = one device program per step
    (pp_batch_run with one instance), "calls" = one C call per operation;
    layer_ops 0 builds the program with every sub-layer as gate launches."""
    from paper_2512_12094_amd import _lib as L
    from paper_2512_12094_amd import driver
    import torch
    layers = driver.heisenberg_layers(prog)
    dp = None
    if mode == "program":
        L.pp_set_layer_ops(layer_ops)
        try:
            dp = driver.DeviceProgram(prog) if layer_ops != 1 else driver.device_program(prog)
        finally:
            L.pp_set_layer_ops(1)
    totals = dict(propagated=0, merged=0, anticommuting=0, appended=0, merge_in=0,
                  merge_out=0, gate_key_reads=0, gate_coef_rw=0)
    kern = {k: [0, 0.0] for k in L.KERNELS}
    L.pp_profile(None, int(profile))
    e = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ps = driver.PauliSet.from_program(prog, group, stream, alloc)
        if mode == "program":
            e = float(L.pp_batch_run([ps.h], [dp.h], stream)[0])
        else:
            driver.run_layers(ps, layers)
            e = ps.expectation(prog.bloch)
        wc = L.pp_work_counters(ps.h)
        for k in totals:
            totals[k] += wc[k]
        if profile:
            for k, (n, ms) in L.pp_profile_read(ps.h).items():
                kern[k][0] += n
                kern[k][1] += ms
        ps.close()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    L.pp_profile(None, 0)
    if dp is not None and layer_ops != 1:
        dp.close()
    return wall, totals, kern, e


MERGE_KINDS = ("merge_narrow", "merge_wide1", "merge_wide2", "part_hist", "part_scan",
               "part_scatter", "part_agg",
               "merge_collect")


def merge_pass(stream, alloc, log2n, dup=32):
    """Exact merge of 2^log2n records: random weight <= 8 Z_32 strings, each
    emitted in `dup` random rotations (Algorithm 1 step 1 on that stream).
    The duration is the sum of the merge kernels' HIP-event intervals (each
    kernel timed on the library's stream, the launch gaps between them
    excluded); `span_ms` is the interval from the first merge kernel's start
    to the last one's end, gaps included."""
    from paper_2512_12094_amd import _lib as L
    from paper_2512_12094_amd import workloads as W
    import torch
    x, z, c = W.merge_stress_records(log2n, dup, seed=7)
    L.pp_profile(None, True)
    torch.cuda.synchronize()
    h = L.pp_create(32, "Zn", x.reshape(-1, 1), z.reshape(-1, 1), c, stream, alloc)
    prof = L.pp_profile_read(h)
    wc = L.pp_work_counters(h)
    st = L.pp_merge_stats(h)
    L.pp_destroy(h)
    L.pp_profile(None, False)
    ms = sum(prof[k][1] for k in MERGE_KINDS)
    nbytes = merge_bytes(wc)
    return dict(records=int(wc["merge_in"]), representatives=int(wc["merge_out"]),
                rotations_per_string=dup, ms=round(ms, 4),
                kernels_ms={k: round(prof[k][1], 4) for k in MERGE_KINDS if prof[k][0]},
                records_per_s=wc["merge_in"] / (ms * 1e-3),
                sort_keys_per_s=wc["merge_in"] / (ms * 1e-3),
                algorithmic_bytes=int(nbytes),
                algorithmic_GBs=round(nbytes / (ms * 1e-3) / 1e9, 1),
                frac_of_hbm=round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                partitioned=st)


def prefix(prog, k):
    """The first k sub-layers of a program in Heisenberg order (the last k
    of its time order): a bounded sample of the same circuit."""
    from paper_2512_12094_amd import workloads as W
    k = min(k, len(prog.sublayers))
    return W.Program(f"{prog.name}[:{k}]", prog.n, prog.group, prog.obs,
                     prog.sublayers[len(prog.sublayers) - k:], prog.bloch, dict(prog.meta))


def gate_scale_leg(stream, alloc):
    """The gate kernel where it is not latency-bound: a Z_32 XXZ ring with
    theta 0.2 and eps 1e-6, weight <= 12, 5 steps (the set grows to
    8.4 x 10^6 representatives).  One device program; every gate launch
    timed (HIP events around each run of back-to-back launches); bytes by
    the same model as the headline roofline."""
    from paper_2512_12094_amd import _lib as L
    from paper_2512_12094_amd import driver
    from paper_2512_12094_amd import workloads as W
    import torch
    prog = W.xxz_ring(32, 5, 0.2, 1.5, eps=1e-6, wmax=12, obs=W.sum_ring_pairs(32, "X"),
                      name="ring32_scale")
    dp = driver.device_program(prog)
    out = None
    for rep in range(2):                       # the first run warms the allocator
        L.pp_profile(None, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ps = driver.PauliSet.from_program(prog, None, stream, alloc)
        L.pp_batch_run([ps.h], [dp.h], stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        L.pp_profile(None, 0)
        wc = L.pp_work_counters(ps.h)
        prof = L.pp_profile_read(ps.h)
        n_final = L.pp_num_terms(ps.h)
        ps.close()
        gate_n, gate_ms = prof["gate"]
        gb = gate_bytes(wc)
        out = dict(workload="Z_32 XXZ ring, theta 0.2, Delta 1.5, eps 1e-6, weight <= 12, 5 steps",
                   final_representatives=int(n_final), units=wc["propagated"] + wc["merged"],
                   wall_s=round(wall, 4), value=(wc["propagated"] + wc["merged"]) / wall,
                   unit="terms/s", gate_launches=gate_n, gate_ms=round(gate_ms, 3),
                   gate_algorithmic_GBs=round(gb / (gate_ms * 1e-3) / 1e9, 1),
                   gate_frac_of_hbm=round(gb / (gate_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))
    return out


def ising_layers_leg(stream, alloc, n=12, layers=(2, 4, 6, 8, 10), dt=0.25):
    """Sec. IV's tilted-field Ising ring (g_x = 1.4, g_z = 0.9045, O = Z at the
    middle site), untruncated: final set size and time per propagation
    against the number of Trotter layers, merged after every sub-layer,
    merged after every full layer (the paper's schedule), and plain PP."""
    from paper_2512_12094_amd import _lib as L
    from paper_2512_12094_amd import driver
    from paper_2512_12094_amd import workloads as W
    import torch
    rows = []
    for nl in layers:
        row = dict(layers=nl)
        for mode in ("sublayer", "layer", "plain"):
            prog = W.tilted_ising_ring(n, nl, dt, merge="layer" if mode == "layer" else "sublayer")
            group = "none" if mode == "plain" else None
            dp = driver.device_program(prog)
            best = None
            for rep in range(2):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ps = driver.PauliSet.from_program(prog, group, stream, alloc)
                L.pp_batch_run([ps.h], [dp.h], stream)
                torch.cuda.synchronize()
                wall = time.perf_counter() - t0
                terms = L.pp_num_terms(ps.h)
                ps.close()
                best = wall if best is None else min(best, wall)
            dp.close()
            row[mode] = dict(terms=int(terms), ms=round(best * 1e3, 3))
        rows.append(row)
    neck = sum(4 ** math.gcd(j, n) for j in range(1, n + 1)) // n
    return dict(workload=f"tilted-field Ising ring n={n}, dt={dt}, untruncated",
                necklaces=neck, rows=rows)


def ising_family_leg(stream, alloc, ns=range(3, 21), max_layers=10, cap=1 << 26,
                     budget_s=8.0, dt=0.25, max_entries=1 << 29):
    """Fig. 2 / Supp. Fig. 1 across n: the tilted-field Ising ring of Sec. IV
    (O = Z at the middle site, untruncated, merged after every Trotter layer)
    for n = 3..20, set size and time per propagation against the number of
    layers, next to plain PP on the same circuit.  A series stops once its set
    passes `cap` terms, a propagation takes longer than `budget_s`, or its
    store would need more than `max_entries` entries (the error is kept)."""
    from paper_2512_12094_amd import _lib as L
    from paper_2512_12094_amd import driver
    from paper_2512_12094_amd import workloads as W
    import torch
    rows = []
    for n in ns:
        row = dict(n=n, necklaces=sum(4 ** math.gcd(j, n) for j in range(1, n + 1)) // n)
        for mode in ("symmetry", "plain"):
            series = []
            for nl in range(1, max_layers + 1):
                prog = W.tilted_ising_ring(n, nl, dt, merge="layer")
                dp = driver.device_program(prog)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ps = driver.PauliSet.from_program(prog, "none" if mode == "plain" else None,
                                                  stream, alloc)
                L.pp_set_max_terms(ps.h, max_entries)
                stop = None
                try:
                    L.pp_batch_run([ps.h], [dp.h], stream)
                except L.PPError as e:
                    stop = f"{nl} layers: {e}"
                torch.cuda.synchronize()
                wall = time.perf_counter() - t0
                terms = L.pp_num_terms(ps.h)
                ps.close()
                dp.close()
                if stop:
                    break
                series.append((nl, int(terms), round(wall * 1e3, 3)))
                if terms > cap or wall > budget_s:
                    break
            row[mode] = dict(layers=[a for a, _, _ in series], terms=[b for _, b, _ in series],
                             ms=[c for _, _, c in series])
            if stop:
                row[mode]["stopped"] = stop
        sat = [t for t in row["symmetry"]["terms"]]
        row["saturated"] = bool(sat) and max(sat) == row["necklaces"] - 1
        assert max(sat) <= row["necklaces"] - 1, (n, max(sat))
        rows.append(row)
        print(f"[ising family] n={n} sym {row['symmetry']['terms'][-1]} terms at "
              f"{row['symmetry']['layers'][-1]} layers", file=sys.stderr, flush=True)
    torch.cuda.empty_cache()                  # the largest stores are not kept for later legs
    return dict(workload=f"tilted-field Ising ring n={ns[0]}..{ns[-1]}, dt={dt}, untruncated, "
                         f"merged per Trotter layer, up to {max_layers} layers, {cap} terms or "
                         f"a store of {max_entries} entries", rows=rows)


def batched_leg(stream, alloc, count, cap_terms):
    """The batched ring workload at full depth (every instance's whole
    program).  A first pass runs every instance alone with a store limit of
    `cap_terms` entries and keeps the instances that finish within it (the
    others, listed, would need more); on those: one batched run (FP64), the
    same batched with FP32 coefficients (largest relative deviation of its
    expectations from FP64), and a loop of single-instance runs, all timed
    from creating each set from its observable."""
    from paper_2512_12094_amd import _lib as L
    from paper_2512_12094_amd import driver
    from paper_2512_12094_amd import workloads as W
    import torch
    allp = W.config4()[:count]
    keep, excluded = [], []
    for p in allp:
        dp = driver.device_program(p)
        ps = driver.PauliSet.from_program(p, None, stream, alloc)
        L.pp_set_max_terms(ps.h, cap_terms)
        try:
            L.pp_batch_run([ps.h], [dp.h], stream)
            keep.append(p)
        except L.PPError:
            excluded.append(dict(name=p.name, n=p.n, sublayers=len(p.sublayers)))
        ps.close()
        dp.close()
    print(f"[bench] batched: {len(keep)} of {len(allp)} instances fit {cap_terms} entries",
          file=sys.stderr, flush=True)
    dps = [driver.device_program(p) for p in keep]

    def solo_loop():
        es, units = [], 0
        for p, dp in zip(keep, dps):
            ps = driver.PauliSet.from_program(p, None, stream, alloc)
            es.append(float(L.pp_batch_run([ps.h], [dp.h], stream)[0]))
            wc = L.pp_work_counters(ps.h)
            units += wc["propagated"] + wc["merged"]
            ps.close()
        return es, units

    def batch(dtype="f64"):
        sets = [driver.PauliSet.from_program(p, None, stream, alloc, dtype) for p in keep]
        e = L.pp_batch_run([s.h for s in sets], [d.h for d in dps], stream)
        units = 0
        for s in sets:
            wc = L.pp_work_counters(s.h)
            units += wc["propagated"] + wc["merged"]
            s.close()
        return [float(v) for v in e], units

    out = {}
    for name, fn in (("batched", batch), ("batched_f32", lambda: batch("f32")),
                     ("per_instance", solo_loop)):
        if name != "per_instance":
            fn()                               # warm (graph capture, allocator)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        es, units = fn()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out[name] = dict(value=units / wall, unit="terms/s", wall_s=round(wall, 4), units=units)
        out[name + "_e"] = es
    e32 = out.pop("batched_f32_e")
    same = sum(a == b for a, b in zip(out.pop("per_instance_e"), out["batched_e"]))
    e64 = out.pop("batched_e")
    out["batched_f32"]["max_rel_dev_from_f64"] = max(
        abs(a - b) / max(abs(b), 1e-300) for a, b in zip(e32, e64))
    out["batched_f32"]["max_abs_dev_over_n"] = max(
        abs(a - b) / p.n for a, b, p in zip(e32, e64, keep))
    out.update(instances=len(allp), full_depth_completed=len(keep),
               excluded_over_store_limit=len(excluded), store_limit_entries=cap_terms,
               excluded_n=sorted({e["n"] for e in excluded}),
               gates=sum(p.n_gates for p in keep),
               speedup=round(out["batched"]["value"] / out["per_instance"]["value"], 3),
               bitwise_equal_expectations=f"{same}/{len(keep)}",
               knobs=L.pp_get_tuning())
    for d in dps:
        d.close()
    return out, keep


def served_leg(stream, alloc, count, cap_terms, seconds, seed=5):
    """Continuous batching of the mixed job stream at full depth (config 5:
    rings and all-to-all Heisenberg jobs), on its first `count` jobs.
    1. Per-instance pass: every job alone (one-instance program path) with a
       store limit of 4 x cap_terms entries; the jobs that finish within it
       are served below (the others, listed by kind, need more), their
       device-tracked peak store sizes seed the estimator, and their summed
       wall time is the per-instance loop's.
    2. Burst: those jobs all arriving at once (the capacity).
    3. Poisson arrivals at 0.8 x that rate, for at most `seconds`.
    p50 / p99 latency over the jobs served."""
    from paper_2512_12094_amd import _lib as L
    from paper_2512_12094_amd import driver
    from paper_2512_12094_amd import serve
    from paper_2512_12094_amd import workloads as W
    import numpy as np
    import torch
    jobs = W.config5(count=count)              # the same first jobs as the full stream
    torch.cuda.empty_cache()                   # what earlier legs left cached
    free, _ = torch.cuda.mem_get_info()
    budget = 0.8 * free
    est = serve.Estimator(cap_terms=cap_terms)
    ok, over = [], []
    wall_solo, units_solo = 0.0, 0
    for j in jobs:
        dp = driver.device_program(j.program)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ps = driver.PauliSet.from_program(j.program, None, stream, alloc)
        L.pp_set_max_terms(ps.h, 4 * cap_terms)
        try:
            L.pp_batch_run([ps.h], [dp.h], stream)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            wc = L.pp_work_counters(ps.h)
            wall_solo += dt
            units_solo += wc["propagated"] + wc["merged"]
            est.observe(j.program, L.pp_peak_terms(ps.h))
            ok.append(j)
        except L.PPError:
            over.append(j)
        ps.close()
        dp.close()
    print(f"[bench] served: {len(ok)} of {len(jobs)} jobs fit {4 * cap_terms} entries",
          file=sys.stderr, flush=True)
    eng = serve.GpuEngine(stream, alloc, steps_per_iter=16)

    def run(js, label, budget_s=None):
        srv = serve.Server(eng, budget, estimator=est)
        ended = [0]

        def progress(kind, i, used):
            if kind in ("finish", "reject"):
                ended[0] += 1
                if ended[0] % 100 == 0:
                    print(f"[bench] served ({label}): {ended[0]}/{len(js)} jobs ended",
                          file=sys.stderr, flush=True)

        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = srv.run(js, on_event=progress, time_budget=budget_s)
        torch.cuda.synchronize()
        return res, time.perf_counter() - t0

    run([W.Job(0.0, j.program) for j in ok[:32]], "warm")
    burst, wall_b = run([W.Job(0.0, j.program) for j in ok], "burst")
    burst_s = serve.summarize(burst, wall_b)
    rate = 0.8 * len(ok) / wall_b
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=len(ok)))
    timed = [W.Job(float(a), j.program) for a, j in zip(t, ok)]
    res, wall = run(timed, "Poisson", seconds)
    summ = serve.summarize(res, wall)
    per = units_solo / wall_solo if wall_solo else None
    summ.update(workload=f"config 5 at full depth, the first {count} of its 2000 jobs (Poisson "
                         "arrivals of 70% Z_n rings and 30% S_n all-to-all jobs)",
                jobs_fitting_store_limit=len(ok), store_limit_entries=4 * cap_terms,
                over_limit_kinds=sorted({f"{j.program.group} n={j.program.n}" for j in over}),
                over_limit_jobs=len(over), time_budget_s=seconds,
                arrival_rate_per_s=round(rate, 2),
                burst=dict(jobs=len(ok), completed=burst_s["completed"],
                           terms_per_s=burst_s["terms_per_s"], wall_s=round(wall_b, 4),
                           p99_s=burst_s["p99_s"]),
                per_instance=dict(terms_per_s=per, wall_s=round(wall_solo, 4)),
                burst_vs_per_instance=round(burst_s["terms_per_s"] / per, 3) if per else None,
                hbm_budget_GB=round(budget / 1e9, 1))
    return summ, timed


def c3_leg(stream, alloc, k=2):
    """Config 3 (S_64 all-to-all Heisenberg, 2016 pair rotations per
    sub-layer, damping p = 1e-3, eps = 1e-5) over its first k sub-layers in
    Heisenberg order, FP64 and FP32 coefficients: terms/s, the expectation,
    and the FP32 coefficients' deviation from FP64 per decade.  Then the
    first k + 1 sub-layers once more with the store allowed 2^31 - 1
    entries, which reports how many entries the next sub-layer needs."""
    from paper_2512_12094_amd import _lib as L
    from paper_2512_12094_amd import driver
    from paper_2512_12094_amd import workloads as W
    import torch
    c3 = W.config3()
    prog = prefix(c3, k)
    dp = driver.device_program(prog)
    res = {}
    for dtype in ("f64", "f32"):
        best = None
        for rep in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ps = driver.PauliSet.from_program(prog, None, stream, alloc, dtype)
            e = float(L.pp_batch_run([ps.h], [dp.h], stream)[0])
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            wc = L.pp_work_counters(ps.h)
            peak = L.pp_peak_terms(ps.h)
            terms = ps.as_dict()
            ps.close()
            best = wall if best is None else min(best, wall)
        units = wc["propagated"] + wc["merged"]
        res[dtype] = dict(value=units / best, unit="terms/s", wall_s=round(best, 4), units=units,
                          expectation=e, peak_entries=peak, representatives=len(terms))
        res[dtype + "_terms"] = terms
    t64, t32 = res.pop("f64_terms"), res.pop("f32_terms")
    scale = max(abs(v) for v in t64.values())
    by_dec = {}
    for key, b in t64.items():
        if key in t32 and b != 0.0:
            dec = int(math.floor(math.log10(abs(b))))
            by_dec[dec] = max(by_dec.get(dec, 0.0), abs(t32[key] - b) / abs(b))
    res["f32_vs_f64"] = dict(expectation_rel=abs(res["f32"]["expectation"] - res["f64"]["expectation"])
                             / max(abs(res["f64"]["expectation"]), 1e-300),
                             coef_rel_by_decade={str(k2): v for k2, v in sorted(by_dec.items())},
                             max_abs_over_max_coef=max(abs(t32.get(k2, 0.0) - v)
                                                       for k2, v in t64.items()) / scale)
    dp.close()
    nxt = prefix(c3, k + 1)
    dpn = driver.device_program(nxt)
    ps = driver.PauliSet.from_program(nxt, None, stream, alloc)
    L.pp_set_max_terms(ps.h, (1 << 31) - 1)
    try:
        L.pp_batch_run([ps.h], [dpn.h], stream)
        res["next_sublayer"] = dict(fits=True, peak_entries=L.pp_peak_terms(ps.h))
    except L.PPError as ex:
        res["next_sublayer"] = dict(fits=False, peak_entries=L.pp_peak_terms(ps.h),
                                    message=str(ex)[:160])
    ps.close()
    dpn.close()
    res.update(workload=f"config 3, first {k} of {len(c3.sublayers)} sub-layers (Heisenberg "
                        "order); the full depth needs more entries inside sub-layer "
                        f"{k + 1} than a store indexes (2^31)" if not res["next_sublayer"]["fits"]
               else f"config 3, first {k} sub-layers")
    return res


# ---------------------------------------------------------------------------
# CPU baselines of the batched and served forms (oracle, host cores)
# ---------------------------------------------------------------------------
def _oracle_job(args):
    """Worker: Algorithm 1 for one program on the oracle, stopping after the
    gate at which the wall clock passes `deadline` (time.time()).  Returns
    (work units done, seconds, finished)."""
    prog, deadline = args
    from oracle import oracle as O
    t0 = time.perf_counter()
    o = O.Oracle(prog.n, prog.group, prog.meta.get("lx", 0), prog.meta.get("perms"))
    for (x, z, c) in prog.obs:
        o.add(x, z, c)
    o.merge()
    finished = True
    for sub in reversed(prog.sublayers):
        if sub.p > 0:
            o.damp(sub.p)
        for g in reversed(sub.gates):
            if time.time() > deadline:
                finished = False
                break
            o.apply_gate(g.x, g.z, g.theta, sub.eps, sub.wmax)
        if not finished:
            break
        if getattr(sub, "merge", True):
            o.merge()
        o.truncate(sub.eps, sub.wmax)
    if finished:
        o.expectation(prog.bloch)
    prop, merged = o.counters()
    return prop + merged, time.perf_counter() - t0, finished


def _host_program(prog):
    """The program without the device objects cached on it (they do not
    cross a process boundary)."""
    import dataclasses
    return dataclasses.replace(prog, meta={k: v for k, v in prog.meta.items()
                                           if not k.startswith("_")})


def cpu_pool_baseline(progs, seconds, workers):
    """The oracle over the batched instances on `workers` host processes,
    each instance until `seconds` have passed (a bounded sample)."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        pool.map(abs, range(workers))          # workers started before the clock
        deadline = time.time() + seconds
        t0 = time.perf_counter()
        out = pool.map(_oracle_job, [(_host_program(p), deadline) for p in progs[:workers]])
    wall = time.perf_counter() - t0
    units = sum(u for u, _, _ in out)
    return dict(value=units / wall, unit="terms/s", cores=workers, kind="oracle",
                sample=f"the first {len(out)} batched instances, one per process, each for at "
                       f"most {seconds:.0f} s ({sum(d for _, _, d in out)} finished; {units} "
                       f"terms in {wall:.1f} s)")


def cpu_served_baseline(timed_jobs, seconds, workers):
    """The served job stream on the oracle: `workers` host processes take
    the jobs FIFO at their arrival times, each job allowed what is left of
    `seconds`; latency = (time its result was ready) - arrival, over the jobs
    that finished."""
    import multiprocessing as mp
    import numpy as np
    ctx = mp.get_context("spawn")
    ready, handles, errors = [], [], []
    progs = [_host_program(j.program) for j in timed_jobs]
    with ctx.Pool(workers) as pool:
        pool.map(abs, range(workers))          # workers started before the clock
        deadline = time.time() + seconds
        t0 = time.perf_counter()
        for j, prog in zip(timed_jobs, progs):
            now = time.perf_counter() - t0
            if j.arrival > seconds or now > seconds:
                break
            if j.arrival > now:
                time.sleep(j.arrival - now)
            cb = (lambda r, a=j.arrival: ready.append((a, time.perf_counter() - t0, r)))
            handles.append(pool.apply_async(_oracle_job, ((prog, deadline),), callback=cb,
                                            error_callback=errors.append))
        for h in handles:
            h.wait()
    if errors:
        raise RuntimeError(f"oracle worker failed: {errors[0]!r}")
    wall = time.perf_counter() - t0
    units = sum(r[0] for _, _, r in ready)
    lat = np.array([f - a for a, f, r in ready if r[2]])
    return dict(value=units / wall, unit="terms/s", cores=workers, kind="oracle",
                jobs_submitted=len(handles), jobs_finished=int(lat.size),
                p50_s=float(np.percentile(lat, 50)) if lat.size else None,
                p99_s=float(np.percentile(lat, 99)) if lat.size else None,
                sample=f"the served job stream's first {len(handles)} arrivals on {workers} "
                       f"oracle processes (FIFO) for {seconds:.0f} s")


def pmc_traffic(bytes_launches, name="k_layer_c2_z32_pmc.json"):
    """HBM bytes per launch (per pass, for the merge summary) from a
    committed rocprofv3 counter summary, when it was taken on the kernel
    sources as they are now."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None, "no counter summary"
    with open(path) as f:
        pmc = json.load(f)
    h = hashlib.sha256()
    for name in pmc["sources"]:
        with open(os.path.join(ROOT, name), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != pmc["sources_sha256"]:
        return None, "kernel sources changed since the counters were taken"
    return (pmc["fetch_kib_per_launch"] * pmc["fetch_scale"] +
            pmc["write_kib_per_launch"] * pmc["write_scale"]) * 1024.0, pmc["command"]


def cpu_baseline(prog, seconds):
    from oracle import oracle as O
    r = O.run_program(prog, keep_terms=False, time_budget=seconds)
    units = r.propagated + r.merged
    return dict(value=units / r.wall, unit="terms/s", cores=1, kind="oracle",
                sample=f"first {r.sublayers_done} of {len(prog.sublayers)} sub-layers of the "
                       f"same workload ({units} terms in {r.wall:.1f} s, one thread)")


def host_info():
    info = dict(nproc=os.cpu_count())
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                info["cpu"] = line.split(":", 1)[1].strip()
    except Exception:
        pass
    return info


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); sharding the "
              "term set by representative hash, with an all-to-all per layer, is not "
              "implemented.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2512_12094_amd import _lib as L
    from paper_2512_12094_amd import workloads as W
    L.lib()
    torch.cuda.set_device(0)
    stream_obj = torch.cuda.Stream()
    stream = int(stream_obj.cuda_stream)
    alloc = L.TorchAllocator(0)
    prog = W.config2()

    from paper_2512_12094_amd import autotune
    tuned_single = autotune.apply(autotune.class_key("single", "Zn", 32))
    with torch.cuda.stream(stream_obj):
        if args.copy_calibration:
            a = torch.empty(64 << 20, dtype=torch.float32, device="cuda")   # 256 MiB
            b = torch.empty_like(a)
            for _ in range(3):
                b.copy_(a)
            torch.cuda.synchronize()
            print(json.dumps({"copy_calibration_bytes_each_way": a.numel() * 4}),
                  file=sys.stderr, flush=True)
        run_steps(prog, "Zn", args.warmup, stream, alloc, False)
        print(f"[bench] warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)
        # timed region: HIP events on the library's stream around every
        # args.event_every-th launch of each kernel kind
        wall, tot, kern, e = run_steps(prog, "Zn", args.steps, stream, alloc, args.event_every)
        print(f"[bench] timed {args.steps} steps in {wall:.3f} s", file=sys.stderr, flush=True)
        # the same steps without events, and through one C call per operation
        wall_np, _, _, _ = run_steps(prog, "Zn", args.steps, stream, alloc, 0)
        wall_calls, _, _, _ = run_steps(prog, "Zn", args.steps, stream, alloc, False,
                                        mode="calls")
        units = tot["propagated"] + tot["merged"]
        value = units / wall
        # the apply step (Algorithm 1 step 2a): one layer op per sub-layer
        # (k_layer_scatter + k_layer_apply), gate launches where a sub-layer
        # has no layer op; each kind's average launch from the sampled events
        from paper_2512_12094_amd import driver
        info = L.pp_program_info(driver.device_program(prog).h)
        layer_ops = info["layer_ops"]
        gate_ops = info["gate_launches"] - layer_ops
        avg = {k: (kern[k][1] * 1e-3 / kern[k][0] if kern[k][0] else 0.0)
               for k in ("gate", "layer_scatter", "layer_apply")}
        op_s = avg["layer_scatter"] + avg["layer_apply"]          # one layer op
        step_apply_s = layer_ops * op_s + gate_ops * avg["gate"]
        gb = gate_bytes(tot) / args.steps                          # per propagation
        apply_ops = layer_ops + gate_ops
        bpl = gb / max(apply_ops, 1)
        avg_s = step_apply_s / max(apply_ops, 1)
        roof = dict(bound="hbm",
                    kernel="apply step: k_layer_scatter + k_layer_apply, one launch pair per "
                           "sub-layer (its 32 rotations)" if layer_ops else "k_gate",
                    achieved=round(bpl / avg_s / 1e9, 2) if avg_s else None,
                    peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(bpl / avg_s / 1e9 / HBM_PEAK_GBS, 5) if avg_s else None,
                    traffic=None,
                    byte_model="per term-gate: 16W key per live term and rotation, 16 B "
                               "coefficient read+write per anticommuting term, 16W+8 B per "
                               "appended child",
                    avg_launch_us=round(avg_s * 1e6, 3),
                    avg_us={k: round(v * 1e6, 3) for k, v in avg.items() if v},
                    timed_launches={k: kern[k][0] for k in avg if kern[k][0]},
                    launches_per_step=dict(layer_ops=layer_ops, gate_launches=gate_ops),
                    bytes_per_launch=round(bpl, 1),
                    rotations_per_launch=round(prog.n_gates / max(apply_ops, 1), 3),
                    est_kernel_ms_per_step=round(step_apply_s * 1e3, 3))
        kernels = {k: dict(launches=n, ms=round(ms, 3)) for k, (n, ms) in kern.items() if n}
        # the same propagation with every sub-layer as fused gate launches
        L.pp_set_layer_ops(0)
        prog_g = W.config2()
        L.pp_set_layer_ops(1)
        wall_gates, _, kern_g, e_g = run_steps(prog_g, "Zn", args.steps, stream, alloc, 0,
                                               layer_ops=0)
        variants = dict(ms_per_step_without_events=round(wall_np / args.steps * 1e3, 3),
                        ms_per_step_one_call_per_op=round(wall_calls / args.steps * 1e3, 3),
                        ms_per_step_gate_launches=round(wall_gates / args.steps * 1e3, 3),
                        gate_launches_same_expectation=e_g == e)
        plain = None
        if not args.no_plain:
            run_steps(prog, "none", 1, stream, alloc, False)
            pw, ptot, pkern, pe = run_steps(prog, "none", max(1, args.steps // 2), stream,
                                            alloc, False)
            psteps = max(1, args.steps // 2)
            plain = dict(value=(ptot["propagated"] + ptot["merged"]) / pw, unit="terms/s",
                         ms_per_step=round(pw / psteps * 1e3, 3),
                         terms_per_step=(ptot["propagated"] + ptot["merged"]) // psteps,
                         expectation=pe)
            print(f"[bench] plain PP done", file=sys.stderr, flush=True)
        dihedral = None
        if not args.no_dihedral:
            run_steps(prog, "Dn", 1, stream, alloc, False)
            dsteps = max(1, args.steps // 2)
            dw, dtot, _, de = run_steps(prog, "Dn", dsteps, stream, alloc, False)
            dihedral = dict(value=(dtot["propagated"] + dtot["merged"]) / dw, unit="terms/s",
                            ms_per_step=round(dw / dsteps * 1e3, 3),
                            terms_per_step=(dtot["propagated"] + dtot["merged"]) // dsteps,
                            expectation=de)
            print(f"[bench] dihedral done", file=sys.stderr, flush=True)
        traffic, traffic_src = pmc_traffic(None, "k_layer_c2_z32_pmc.json")
        roof["traffic"] = round(traffic, 1) if traffic is not None else None
        roof["traffic_unit"] = ("HBM bytes per layer op, k_layer_scatter + k_layer_apply "
                                "(rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled)")
        roof["traffic_source"] = traffic_src
        mp = roof_merge = None
        if not args.no_merge_pass:
            merge_pass(stream, alloc, args.merge_log2n)            # warm
            mp = merge_pass(stream, alloc, args.merge_log2n)
            keep = ("records", "rotations_per_string", "representatives", "ms",
                    "records_per_s", "algorithmic_GBs", "frac_of_hbm")
            mp["other_duplicate_factors"] = [
                {k: v for k, v in merge_pass(stream, alloc, args.merge_log2n, d).items()
                 if k in keep} for d in (1, 4)]
            mp["other_sizes"] = []
            for lg in args.merge_more:
                merge_pass(stream, alloc, lg)                      # warm the allocator
                mp["other_sizes"].append({k: v for k, v in merge_pass(stream, alloc, lg).items()
                                          if k in keep})
            mtraffic, msrc = pmc_traffic(None, "k_merge_stress_2p24_pmc.json")
            roof_merge = dict(bound="hbm", kernel="merge pass (k_part_hist, k_part_scan, "
                              "k_part_scatter, k_part_agg, k_merge_collect)",
                              achieved=mp["algorithmic_GBs"], peak=HBM_PEAK_GBS, unit="GB/s",
                              frac=mp["frac_of_hbm"],
                              traffic=round(mtraffic, 1) if mtraffic is not None else None,
                              traffic_unit="HBM bytes per pass of 2^24 records (rocprofv3 "
                                           "FETCH_SIZE + WRITE_SIZE, scaled)",
                              traffic_source=msrc, algorithmic_bytes=mp["algorithmic_bytes"],
                              byte_model="(16W + 8) B per record read + (16W + 8) B per "
                                         "representative written")
            print(f"[bench] merge pass done", file=sys.stderr, flush=True)
        ising = None
        if not args.no_ising:
            ising = ising_layers_leg(stream, alloc)
        ising_family = None
        if not args.no_ising_family:
            ising_family = ising_family_leg(stream, alloc)
            print(f"[bench] Ising layers leg done", file=sys.stderr, flush=True)
        scale = None
        if not args.no_scale:
            scale = gate_scale_leg(stream, alloc)
            print(f"[bench] gate-at-scale leg done", file=sys.stderr, flush=True)
        c3 = None
        if not args.no_c3:
            c3 = c3_leg(stream, alloc)
            print(f"[bench] all-to-all leg done", file=sys.stderr, flush=True)
        batched = served = None
        batch_progs = served_jobs = None
        if not args.no_batched:
            tuned_batch = autotune.apply(autotune.class_key("batch", "Zn"))
            batched, batch_progs = batched_leg(stream, alloc, args.batch_count,
                                               args.batch_cap_terms)
            batched["tuned"] = tuned_batch is not None
            print(f"[bench] batched leg done", file=sys.stderr, flush=True)
        if not args.no_served:
            served, served_jobs = served_leg(stream, alloc, args.serve_count,
                                             args.serve_cap_terms, args.serve_seconds)
            print(f"[bench] served leg done", file=sys.stderr, flush=True)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "c2_z32_xxz: Z_32 ring, 20 XXZ Trotter steps (theta 0.05, "
                               "Delta 1.5), O = sum X_i X_{i+1}, eps 1e-4, weight <= 8, "
                               "symmetry PP under translations",
                   "n": 32, "sublayers": 60, "gates": 1920,
                   "terms_per_step": units // args.steps, "expectation": e},
        "plain_pp": plain,
        "dihedral_pp": dihedral,
        "gate_at_scale": scale,
        "ising_layers": ising,
        "ising_family": ising_family,
        "roofline": roof,
        "roofline_merge": roof_merge,
        "kernels": kernels,
        "variants": variants,
        "tuning": {"single": tuned_single, "source": autotune.cache_path()},
        "merge_pass": mp,
        "all_to_all_c3": c3,
        "batched": batched,
        "served": served,
        "host": host_info(),
        "platform": platform.node(),
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prog, args.cpu_seconds)
        workers = max(1, min(16, os.cpu_count() or 1))
        if batch_progs:
            batched["cpu_baseline"] = cpu_pool_baseline(batch_progs, args.cpu_pool_seconds,
                                                        workers)
        if served_jobs:
            served["cpu_baseline"] = cpu_served_baseline(served_jobs, args.cpu_pool_seconds,
                                                         workers)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
