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
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--batch-sublayers", type=int, default=12)
    ap.add_argument("--serve-count", type=int, default=200)
    ap.add_argument("--serve-sublayers", type=int, default=3)
    ap.add_argument("--serve-cap-terms", type=int, default=1 << 24,
                    help="largest estimate a served job may reach (store = 4x)")
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


def run_steps(prog, group, steps, stream, alloc, profile, mode="program"):
    """`steps` propagations; mode "program" = one device program per step
    (pp_batch_run with one instance), "calls" = one C call per operation."""
    from paper_2512_12094_amd import _lib as L
    from paper_2512_12094_amd import driver
    import torch
    layers = driver.heisenberg_layers(prog)
    dp = driver.device_program(prog) if mode == "program" else None
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


def batched_leg(stream, alloc, count, sublayers):
    """Batched ring instances (uneven n, depth, angles, thresholds; each cut
    to its first `sublayers` sub-layers): one batched run against a loop of
    single-instance runs over the same instances, and the batched run with
    FP32 coefficients (largest relative deviation of its expectations from
    the FP64 ones).  All include creating each instance's set from its
    observable."""
    from paper_2512_12094_amd import _lib as L
    from paper_2512_12094_amd import driver
    from paper_2512_12094_amd import workloads as W
    import torch
    progs = [prefix(p, sublayers) for p in W.config4()[:count]]
    dps = [driver.device_program(p) for p in progs]

    def solo_loop():
        es, units = [], 0
        for p, dp in zip(progs, dps):
            ps = driver.PauliSet.from_program(p, None, stream, alloc)
            es.append(float(L.pp_batch_run([ps.h], [dp.h], stream)[0]))
            wc = L.pp_work_counters(ps.h)
            units += wc["propagated"] + wc["merged"]
            ps.close()
        return es, units

    def batch(dtype="f64"):
        sets = [driver.PauliSet.from_program(p, None, stream, alloc, dtype) for p in progs]
        e = L.pp_batch_run([s.h for s in sets], [d.h for d in dps], stream)
        units = 0
        for s in sets:
            wc = L.pp_work_counters(s.h)
            units += wc["propagated"] + wc["merged"]
            s.close()
        return [float(v) for v in e], units

    out = {}
    for name, fn in (("per_instance", solo_loop), ("batched", batch),
                     ("batched_f32", lambda: batch("f32"))):
        fn()                                   # warm (graph capture, allocator)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        es, units = fn()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out[name] = dict(value=units / wall, unit="terms/s", wall_s=round(wall, 4), units=units)
        out[name + "_e"] = es
    e32 = out.pop("batched_f32_e")
    same = sum(a == b for a, b in zip(out.pop("per_instance_e"), out["batched_e"]))
    out["batched_f32"]["max_rel_dev_from_f64"] = max(
        abs(a - b) / max(abs(b), 1e-300) for a, b in zip(e32, out.pop("batched_e")))
    out.update(instances=len(progs), sublayers_each=sublayers,
               gates=sum(p.n_gates for p in progs),
               speedup=round(out["batched"]["value"] / out["per_instance"]["value"], 3),
               bitwise_equal_expectations=f"{same}/{len(progs)}",
               knobs=L.pp_get_tuning())
    return out


def served_leg(stream, alloc, count, sublayers, cap_terms, seed=5):
    """Continuous batching of a mixed job stream (rings and all-to-all
    Heisenberg jobs, each cut to its first `sublayers` sub-layers).  A first,
    untimed pass serves every job once (the estimator learns peak sizes per
    job class; a job whose store would exceed 4 x cap_terms entries is
    rejected and listed).  On the jobs that completed, the leg then times:
    a loop of single-instance runs; serving them all arriving at once (the
    capacity); serving them with Poisson arrivals at 0.8 x that rate (p50 /
    p99 latency)."""
    from paper_2512_12094_amd import _lib as L
    from paper_2512_12094_amd import driver
    from paper_2512_12094_amd import serve
    from paper_2512_12094_amd import workloads as W
    import numpy as np
    import torch
    jobs = [W.Job(0.0, prefix(j.program, sublayers)) for j in W.config5(count=count)]
    free, _ = torch.cuda.mem_get_info()
    budget = 0.8 * free
    est = serve.Estimator(cap_terms=cap_terms)
    eng = serve.GpuEngine(stream, alloc, steps_per_iter=16)

    def run(js, label):
        srv = serve.Server(eng, budget, estimator=est)
        ended = [0]

        def progress(kind, i, used):
            if kind in ("finish", "reject"):
                ended[0] += 1
                if ended[0] % 25 == 0:
                    print(f"[bench] served ({label}): {ended[0]}/{len(js)} jobs ended",
                          file=sys.stderr, flush=True)

        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = srv.run(js, on_event=progress)
        torch.cuda.synchronize()
        return res, time.perf_counter() - t0

    first, _ = run(jobs, "learning")
    done = [j for j, r in zip(jobs, first) if not r.rejected]
    rejected = sorted({f"{j.program.group} n={j.program.n}"
                       for j, r in zip(jobs, first) if r.rejected})

    # single-instance loop over the same jobs
    dps = [driver.device_program(j.program) for j in done]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    units_solo = 0
    for j, dp in zip(done, dps):
        ps = driver.PauliSet.from_program(j.program, None, stream, alloc)
        L.pp_set_max_terms(ps.h, 4 * cap_terms)
        L.pp_batch_run([ps.h], [dp.h], stream)
        wc = L.pp_work_counters(ps.h)
        units_solo += wc["propagated"] + wc["merged"]
        ps.close()
    torch.cuda.synchronize()
    wall_solo = time.perf_counter() - t0

    burst, wall_b = run(done, "burst")
    rate = 0.8 * len(done) / wall_b
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=len(done)))
    timed = [W.Job(float(a), j.program) for a, j in zip(t, done)]
    res, wall = run(timed, "Poisson")
    summ = serve.summarize(res, wall)
    burst_s = serve.summarize(burst, wall_b)
    summ.update(sampled_jobs=len(jobs), sublayers_each=sublayers,
                store_limit_terms=4 * cap_terms, rejected_in_learning_pass=len(jobs) - len(done),
                rejected_kinds=rejected, ring_jobs=sum(j.program.group == "Zn" for j in done),
                arrival_rate_per_s=round(rate, 2),
                burst=dict(terms_per_s=burst_s["terms_per_s"], wall_s=round(wall_b, 4),
                           jobs_per_s=round(len(done) / wall_b, 2), p99_s=burst_s["p99_s"]),
                per_instance=dict(terms_per_s=units_solo / wall_solo, wall_s=round(wall_solo, 4)),
                burst_vs_per_instance=round(burst_s["terms_per_s"] / (units_solo / wall_solo), 3),
                hbm_budget_GB=round(budget / 1e9, 1))
    return summ


def pmc_traffic(bytes_launches, name="k_gate_c2_z32_pmc.json"):
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
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the term set "
              "would shard by representative hash with an all-to-all per layer, which this "
              "build does not implement.", file=sys.stderr)
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
        gate_n, gate_ms = kern["gate"]             # sampled launches and their time
        from paper_2512_12094_amd import driver
        per_step = L.pp_program_info(driver.device_program(prog).h)["gate_launches"]
        gates_run = per_step * args.steps           # every gate op runs once per step
        gb = gate_bytes(tot)
        avg_s = gate_ms * 1e-3 / max(gate_n, 1)
        bpl = gb / gates_run
        bpl_launch = gate_bytes_launch(tot) / gates_run
        roof = dict(bound="hbm", kernel="k_gate", achieved=round(bpl / avg_s / 1e9, 2),
                    peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(bpl / avg_s / 1e9 / HBM_PEAK_GBS, 5), traffic=None,
                    byte_model="per term-gate: 16W key per live term and rotation, 16 B "
                               "coefficient read+write per anticommuting term, 16W+8 B per "
                               "appended child",
                    avg_launch_us=round(avg_s * 1e6, 3), timed_launches=gate_n,
                    launches=gates_run, bytes_per_launch=round(bpl, 1),
                    launch_model=dict(bytes_per_launch=round(bpl_launch, 1),
                                      achieved=round(bpl_launch / avg_s / 1e9, 2),
                                      frac=round(bpl_launch / avg_s / 1e9 / HBM_PEAK_GBS, 5)),
                    rotations_per_launch=round(prog.n_gates / per_step, 3),
                    est_kernel_ms_per_step=round(avg_s * 1e3 * per_step, 3))
        kernels = {k: dict(launches=n, ms=round(ms, 3)) for k, (n, ms) in kern.items() if n}
        variants = dict(ms_per_step_without_events=round(wall_np / args.steps * 1e3, 3),
                        ms_per_step_one_call_per_op=round(wall_calls / args.steps * 1e3, 3))
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
        traffic, traffic_src = pmc_traffic(None)
        roof["traffic"] = round(traffic, 1) if traffic is not None else None
        roof["traffic_unit"] = "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled)"
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
            print(f"[bench] Ising layers leg done", file=sys.stderr, flush=True)
        scale = None
        if not args.no_scale:
            scale = gate_scale_leg(stream, alloc)
            print(f"[bench] gate-at-scale leg done", file=sys.stderr, flush=True)
        batched = served = None
        if not args.no_batched:
            tuned_batch = autotune.apply(autotune.class_key("batch", "Zn"))
            batched = batched_leg(stream, alloc, args.batch_count, args.batch_sublayers)
            batched["tuned"] = tuned_batch is not None
            print(f"[bench] batched leg done", file=sys.stderr, flush=True)
        if not args.no_served:
            served = served_leg(stream, alloc, args.serve_count, args.serve_sublayers,
                                args.serve_cap_terms)
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
        "roofline": roof,
        "roofline_merge": roof_merge,
        "kernels": kernels,
        "variants": variants,
        "tuning": {"single": tuned_single, "source": autotune.cache_path()},
        "merge_pass": mp,
        "batched": batched,
        "served": served,
        "host": host_info(),
        "platform": platform.node(),
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prog, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
