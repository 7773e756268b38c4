"""Autotuner for the library's launch parameters (pp_set_tuning).

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

KNOBS = {
    "gate_items": [1, 2, 4],
    "stream_items": [1, 2, 4, 8],
    "max_blocks": [256, 512, 1024, 2048],
    "graph_steps": [8, 16, 32, 64],
    "gates_per_step": [1, 2, 4, 8, 16],
}
SINGLE_KNOBS = ("gate_items", "stream_items", "max_blocks")
BATCH_KNOBS = tuple(KNOBS)


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
    L.pp_set_tuning(**{k: int(entry["knobs"][k]) for k in KNOBS if k in entry["knobs"]})
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
    best = L.pp_get_tuning()

    def measure(setting):
        L.pp_set_tuning(**setting)
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
    L.pp_set_tuning(**best)
    cache = load_cache(path)
    cache.setdefault(device_name(), {})[key] = dict(
        knobs=best, seconds=best_t, trials=len(trials),
        baseline_seconds=trials[0][1])
    save_cache(cache, path)
    return best
