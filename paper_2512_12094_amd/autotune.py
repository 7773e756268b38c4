"""Autotuner for the library's launch parameters (pp_set_tuning), the
layer op's bucket size and block size (pp_set_layer_tuning) and the
partitioned merge's bucket size and aggregation grid (pp_set_merge_tuning).

A workload class (e.g. "single:Zn:n32" for one-instance programs of Z_n
rings near 32 qubits, "batch:Zn" for batched rings) maps to the knob values
that ran a representative sample fastest on this device.  The search is a
coordinate descent over the knob grid (each knob swept with the others
fixed, two rounds), timing the sample with a device synchronisation on both
sides and taking the median of a few repetitions.  Results persist in a
JSON cache keyed by device name and class; `apply(key)` loads them into the
library before a run.
"""
from __future__ import annotations

import json
import os
import statistics
import time

from . import _lib as L

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tuning.json")

LAUNCH_KNOBS = {
    "gate_items": [1, 2, 4],
    "stream_items": [1, 2, 4, 8],
    "max_blocks": [256, 512, 1024, 2048],
    "graph_steps": [8, 16, 32, 64],
    "gates_per_step": [1, 2, 4, 8, 16],
}
LAYER_KNOBS = {"layer_shift": [6, 7, 8, 9], "layer_block": [256, 512]}
MERGE_KNOBS = {"part_shift": [12, 13, 14, 15], "part_agg_blocks": [0, 512, 1024, 2048]}
KNOBS = {**LAUNCH_KNOBS, **LAYER_KNOBS, **MERGE_KNOBS}
SINGLE_KNOBS = ("gate_items", "stream_items", "max_blocks", "layer_shift", "layer_block")
BATCH_KNOBS = tuple(LAUNCH_KNOBS)
MERGE_PASS_KNOBS = tuple(MERGE_KNOBS)


def get_knobs() -> dict:
    """Every knob's current value."""
    out = dict(L.pp_get_tuning())
    lt = L.pp_get_layer_tuning()
    out.update(layer_shift=lt["bucket_log2"], layer_block=lt["block"])
    mt = L.pp_get_merge_tuning()
    out.update(part_shift=mt[0] if isinstance(mt, (list, tuple)) else mt["bucket_log2"],
               part_agg_blocks=mt[1] if isinstance(mt, (list, tuple)) else mt["agg_blocks"])
    return out


def set_knobs(setting: dict):
    """Sets the knobs named in `setting` (the others keep their values)."""
    launch = {k: int(v) for k, v in setting.items() if k in LAUNCH_KNOBS}
    if launch:
        cur = L.pp_get_tuning()
        L.pp_set_tuning(**{k: int(launch.get(k, cur[k])) for k in LAUNCH_KNOBS})
    if "layer_shift" in setting or "layer_block" in setting:
        L.pp_set_layer_tuning(int(setting.get("layer_shift", 0)), int(setting.get("layer_block", 0)))
    if "part_shift" in setting or "part_agg_blocks" in setting:
        cur = get_knobs()
        L.pp_set_merge_tuning(int(setting.get("part_shift", cur["part_shift"])),
                              int(setting.get("part_agg_blocks", cur["part_agg_blocks"])))


def cache_path() -> str:
    return os.environ.get("PP_TUNING_CACHE", DEFAULT_CACHE)


def device_name() -> str:
    try:
        import torch
        return torch.cuda.get_device_name(0)
    except Exception:
        return "unknown"


def load_cache(path: str | None = None) -> dict:
    path = path or cache_path()
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def save_cache(cache: dict, path: str | None = None):
    path = path or cache_path()
    tmp = path + f".tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def class_key(kind: str, group: str, n: int | None = None) -> str:
    """Workload class: kind ("single" or "batch"), group, qubit bucket."""
    if n is None:
        return f"{kind}:{group}"
    bucket = 16
    while bucket < n:
        bucket *= 2
    return f"{kind}:{group}:n{bucket}"


def apply(key: str, path: str | None = None) -> dict | None:
    """Sets the cached knobs of `key` (if any) and returns them."""
    entry = load_cache(path).get(device_name(), {}).get(key)
    if entry is None:
        return None
    set_knobs({k: v for k, v in entry["knobs"].items() if k in KNOBS})
    return entry["knobs"]


def time_once(run, sync) -> float:
    sync()
    t0 = time.perf_counter()
    run()
    sync()
    return time.perf_counter() - t0


def tune(key: str, run, knobs=BATCH_KNOBS, reps: int = 3, rounds: int = 2,
         sync=None, path: str | None = None, log=print) -> dict:
    """Coordinate descent over `knobs` for the sample `run` (a callable that
    executes the workload once); stores and returns the best setting."""
    if sync is None:
        import torch
        sync = torch.cuda.synchronize
    best = {k: v for k, v in get_knobs().items() if k in knobs}

    def measure(setting):
        set_knobs(setting)
        run()                                   # warm (graph capture, allocation)
        return statistics.median(time_once(run, sync) for _ in range(reps))

    best_t = measure(best)
    trials = [(dict(best), best_t)]
    for _ in range(rounds):
        improved = False
        for k in knobs:
            for v in KNOBS[k]:
                if v == best[k]:
                    continue
                cand = dict(best, **{k: v})
                t = measure(cand)
                trials.append((cand, t))
                if t < best_t * 0.98:
                    best, best_t, improved = cand, t, True
                    log(f"[autotune] {key}: {k}={v} -> {t * 1e3:.2f} ms")
        if not improved:
            break
    set_knobs(best)
    cache = load_cache(path)
    cache.setdefault(device_name(), {})[key] = dict(
        knobs=best, seconds=best_t, trials=len(trials),
        baseline_seconds=trials[0][1])
    save_cache(cache, path)
    return best


def _tune_workloads(path: str | None, log=print) -> dict:
    """Tunes the classes of the ring workloads: one-instance Z_32 programs
    (the 20-step XXZ ring) and batched rings (256 instances of mixed n,
    12 sub-layers each)."""
    import torch
    from . import driver
    from . import workloads as W
    L.lib()
    torch.cuda.set_device(0)
    so = torch.cuda.Stream()
    stream = int(so.cuda_stream)
    alloc = L.TorchAllocator(0)
    out = {}
    with torch.cuda.stream(so):
        prog = W.config2()
        dp = driver.device_program(prog)

        def single():
            ps = driver.PauliSet.from_program(prog, None, stream, alloc)
            L.pp_batch_run([ps.h], [dp.h], stream)
            ps.close()

        out["single:Zn:n32"] = tune(class_key("single", "Zn", 32), single, SINGLE_KNOBS,
                                    path=path, log=log)
        progs = []
        for p in W.config4():
            k = min(12, len(p.sublayers))
            progs.append(W.Program(p.name, p.n, p.group, p.obs, p.sublayers[len(p.sublayers) - k:],
                                   p.bloch, dict(p.meta)))
        dps = [driver.device_program(p) for p in progs]

        def batch():
            sets = [driver.PauliSet.from_program(p, None, stream, alloc) for p in progs]
            L.pp_batch_run([s.h for s in sets], [d.h for d in dps], stream)
            for s in sets:
                s.close()

        out["batch:Zn"] = tune(class_key("batch", "Zn"), batch, BATCH_KNOBS, path=path, log=log)

        x, z, c = W.merge_stress_records(24, 32, seed=7)

        def merge_pass():
            h = L.pp_create(32, "Zn", x.reshape(-1, 1), z.reshape(-1, 1), c, stream, alloc)
            L.pp_destroy(h)

        out["merge:Zn:n32"] = tune(class_key("merge", "Zn", 32), merge_pass, MERGE_PASS_KNOBS,
                                   path=path, log=log)
    return out


if __name__ == "__main__":
    import sys
    print(json.dumps(_tune_workloads(sys.argv[1] if len(sys.argv) > 1 else None)), flush=True)
