"""Comparison rules between the HIP path and the CPU oracle.

* Pauli sets: identical keys (bit-exact integer masks).  When a coefficient
  threshold eps is on, strings whose |c| lies within 1e-9 relative of eps on
  either side are left out of the set comparison.
* FP64 coefficients: |a - b| <= 1e-12 max(|a|, |b|) + 1e-12 max_r |c_r|
  (the absolute floor covers exact cancellations to zero).
* Expectations: |a - b| <= 1e-12 sum_r |c_r| (the scale of the sum's terms).

FP32 coefficient mode against the FP64 oracle:

* coefficients: |a - b| <= 1e-5 max(|a|, |b|) + 2^-21 max_r |c_r|.  The
  relative part is the stated FP32 accuracy; the floor allows 8 FP32
  roundings (unit 2^-24) of terms as large as the largest coefficient,
  which covers cancellations (measured: at most 4.6 such roundings on the
  ring, all-to-all and batched workloads).  `f32_error_report` gives the
  achieved relative error per decade of coefficient magnitude.
* Pauli sets: strings whose |c| lies within that floor of eps (absolute) on
  either side are left out, since FP32 rounding may move them across it.
* Expectations: |a - b| <= 1e-5 sum_r |c_r|.
"""
from __future__ import annotations

REL = 1e-12
BAND = 1e-9
REL32 = 1e-5
FLOOR32 = 2.0 ** -21


def near_threshold(c: float, eps: float, band_abs: float = 0.0) -> bool:
    return eps > 0 and abs(abs(c) - eps) <= max(BAND * eps, band_abs)


def compare_terms(gpu: dict, ref: dict, eps: float = 0.0, rel: float = REL, what: str = "",
                  floor: float | None = None, band_abs: float = 0.0):
    """floor: absolute floor relative to max_r |c_r| (default: rel)."""
    skip = {k for k, v in gpu.items() if near_threshold(v, eps, band_abs)} | \
           {k for k, v in ref.items() if near_threshold(v, eps, band_abs)}
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
    fl = rel if floor is None else floor
    assert worst <= fl * scale, f"{what}: coefficient {wk}: gpu {gpu[wk]!r} oracle {ref[wk]!r}"
    return len(gk), len(skip)


def compare_terms_f32(gpu: dict, ref: dict, eps: float = 0.0, what: str = ""):
    """FP32 coefficient mode against the FP64 oracle (rules above)."""
    scale = max([abs(v) for v in ref.values()] + [0.0])
    return compare_terms(gpu, ref, eps, rel=REL32, what=what, floor=FLOOR32,
                         band_abs=FLOOR32 * scale)


def compare_expectation(a: float, b: float, terms: dict, rel: float = REL, what: str = ""):
    scale = max(1.0, sum(abs(v) for v in terms.values()))
    assert abs(a - b) <= rel * scale, f"{what}: expectation gpu {a!r} oracle {b!r}"


def f32_error_report(gpu: dict, ref: dict) -> dict:
    """Largest relative error |a - b| / |b| of the FP32 coefficients per
    decade of |b| (keys: floor(log10 |b|)), over the strings both sides
    hold; and the largest error in units of 2^-24 max_r |c_r|."""
    import math
    scale = max([abs(v) for v in ref.values()] + [0.0])
    out, worst_units = {}, 0.0
    for k, b in ref.items():
        if k not in gpu or b == 0.0:
            continue
        e = abs(gpu[k] - b)
        dec = int(math.floor(math.log10(abs(b))))
        out[dec] = max(out.get(dec, 0.0), e / abs(b))
        if scale:
            worst_units = max(worst_units, e / (scale * 2.0 ** -24))
    return {"rel_by_decade": dict(sorted(out.items())), "worst_roundings": worst_units}
