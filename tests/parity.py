"""Comparison rules between the HIP path and the CPU oracle.

* Pauli sets: identical keys (bit-exact integer masks).  When a coefficient
  threshold eps is on, strings whose |c| lies within 1e-9 relative of eps on
  either side are left out of the set comparison.
* FP64 coefficients: |a - b| <= 1e-12 max(|a|, |b|) + 1e-12 max_r |c_r|
  (the absolute floor covers exact cancellations to zero).
* Expectations: |a - b| <= 1e-12 sum_r |c_r| (the scale of the sum's terms).
"""
from __future__ import annotations

REL = 1e-12
BAND = 1e-9


def near_threshold(c: float, eps: float) -> bool:
    return eps > 0 and abs(abs(c) - eps) <= BAND * eps


def compare_terms(gpu: dict, ref: dict, eps: float = 0.0, rel: float = REL, what: str = ""):
    skip = {k for k, v in gpu.items() if near_threshold(v, eps)} | \
           {k for k, v in ref.items() if near_threshold(v, eps)}
    gk, rk = set(gpu) - skip, set(ref) - skip
    if gk != rk:
        only_g, only_r = list(gk - rk)[:5], list(rk - gk)[:5]
        raise AssertionError(
            f"{what}: sets differ: {len(gk - rk)} only on GPU (e.g. "
            f"{[(k, gpu[k]) for k in only_g]}), {len(rk - gk)} only in oracle (e.g. "
            f"{[(k, ref[k]) for k in only_r]})")
    scale = max([abs(v) for v in ref.values()] + [0.0])
    worst, wk = 0.0, None
    for k in gk:
        a, b = gpu[k], ref[k]
        err = abs(a - b) - rel * max(abs(a), abs(b))
        if err > worst:
            worst, wk = err, k
    assert worst <= rel * scale, f"{what}: coefficient {wk}: gpu {gpu[wk]!r} oracle {ref[wk]!r}"
    return len(gk), len(skip)


def compare_expectation(a: float, b: float, terms: dict, rel: float = REL, what: str = ""):
    scale = max(1.0, sum(abs(v) for v in terms.values()))
    assert abs(a - b) <= rel * scale, f"{what}: expectation gpu {a!r} oracle {b!r}"
