"""Python side of the CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg import this module.  It wraps ``pp_oracle.cpp`` with
ctypes and runs Algorithm 1 of arXiv:2512.12094 over a
``paper_2512_12094_amd.workloads.Program``:

1. the observable's rows are added up and merged by orbit representative
   (Algorithm 1, step 1);
2. for every sub-layer in Heisenberg order (the time-ordered list walked
   backwards): depolarising damping, then each gate (also walked backwards,
   so that the pass computes U^dag O U exactly), each followed by the exact
   merge of identical strings and the truncation; then the symmetry merge
   (step 2b) and the truncation;
3. the expectation in the symmetric product state (step 3).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pp_oracle.cpp")
_LIB = os.path.join(_HERE, "libpp_oracle.so")

GROUP_CODE = {"none": 0, "Zn": 1, "Sn": 2, "Dn": 3}
TORUS = "T2"   # translations of an lx x ly torus (the width travels separately)
EXPLICIT = "G"  # a group given by its list of qubit permutations

_u64p = ctypes.POINTER(ctypes.c_uint64)
_f64p = ctypes.POINTER(ctypes.c_double)


def build(force: bool = False) -> str:
    """Compile the oracle with the host compiler (no GPU code involved)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        L.orc_create.restype = ctypes.c_void_p
        L.orc_create.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_add_term.argtypes = [ctypes.c_void_p, _u64p, _u64p, ctypes.c_double]
        L.orc_merge.argtypes = [ctypes.c_void_p]
        L.orc_apply_gate.argtypes = [ctypes.c_void_p, _u64p, _u64p, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_int]
        L.orc_damp.argtypes = [ctypes.c_void_p, ctypes.c_double]
        L.orc_truncate.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int]
        L.orc_expectation.restype = ctypes.c_double
        L.orc_expectation.argtypes = [ctypes.c_void_p] + [ctypes.c_double] * 3
        L.orc_size.restype = ctypes.c_size_t
        L.orc_size.argtypes = [ctypes.c_void_p]
        L.orc_export.argtypes = [ctypes.c_void_p, _u64p, _u64p, _f64p]
        L.orc_counters.argtypes = [ctypes.c_void_p, _u64p, _u64p]
        L.orc_canon.argtypes = [ctypes.c_int, ctypes.c_int, _u64p, _u64p, _u64p, _u64p]
        L.orc_canon_torus.argtypes = [ctypes.c_int, ctypes.c_int, _u64p, _u64p, _u64p, _u64p]
        L.orc_create_group.restype = ctypes.c_void_p
        L.orc_create_group.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t]
        L.orc_canon_group.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t,
                                      _u64p, _u64p, _u64p, _u64p]
        L.orc_create_torus.restype = ctypes.c_void_p
        L.orc_create_torus.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_multiply.restype = ctypes.c_int
        L.orc_multiply.argtypes = [ctypes.c_int] + [_u64p] * 6
        L.orc_merge_records.restype = ctypes.c_size_t
        L.orc_merge_records.argtypes = [ctypes.c_int, ctypes.c_int, _u64p, _u64p, _f64p,
                                        ctypes.c_size_t, _u64p, _u64p, _f64p]
        L.orc_exact_sum.restype = ctypes.c_double
        L.orc_exact_sum.argtypes = [_f64p, ctypes.c_size_t]
        L.orc_int_less.restype = ctypes.c_int
        L.orc_int_less.argtypes = [ctypes.c_int] + [_u64p] * 4
        _lib = L
    return _lib


def _words(v: int, W: int):
    return (ctypes.c_uint64 * W)(*[(v >> (64 * w)) & 0xFFFFFFFFFFFFFFFF for w in range(W)])


def _join(ws) -> int:
    return sum(int(w) << (64 * i) for i, w in enumerate(ws))


def _perm_array(perms, n):
    a = np.ascontiguousarray(np.asarray(perms, dtype=np.uint8).reshape(-1, n))
    return a, len(a)


def canon(n: int, group: str, x: int, z: int, lx: int = 0, perms=None):
    """Representative of (x, z); group TORUS needs the torus width lx,
    group EXPLICIT the element list perms (rows of n qubit indices)."""
    W = (n + 63) // 64
    rx, rz = (ctypes.c_uint64 * W)(), (ctypes.c_uint64 * W)()
    if group == EXPLICIT:
        a, m = _perm_array(perms, n)
        lib().orc_canon_group(n, a.ctypes.data, m, _words(x, W), _words(z, W), rx, rz)
    elif group == TORUS:
        lib().orc_canon_torus(lx, n // lx, _words(x, W), _words(z, W), rx, rz)
    else:
        lib().orc_canon(n, GROUP_CODE[group], _words(x, W), _words(z, W), rx, rz)
    return _join(rx), _join(rz)


def multiply(n: int, a, b):
    """(ax, az) * (bx, bz) = i^k (rx, rz); returns (k, rx, rz)."""
    W = (n + 63) // 64
    rx, rz = (ctypes.c_uint64 * W)(), (ctypes.c_uint64 * W)()
    k = lib().orc_multiply(n, _words(a[0], W), _words(a[1], W), _words(b[0], W),
                           _words(b[1], W), rx, rz)
    return k, _join(rx), _join(rz)


def exact_sum(values) -> float:
    v = np.ascontiguousarray(values, dtype=np.float64)
    return lib().orc_exact_sum(v.ctypes.data_as(_f64p), len(v))


def merge_records(n: int, group: str, x, z, c) -> dict:
    """Algorithm 1 step 1 on raw rows: {representative: exact sum of every
    row of its orbit, repeated rows counted as separate addends}.  x, z:
    arrays of shape (m,) or (m, W) of uint64; c: m doubles."""
    W = (n + 63) // 64
    xa = np.ascontiguousarray(np.asarray(x, dtype=np.uint64).reshape(-1, W))
    za = np.ascontiguousarray(np.asarray(z, dtype=np.uint64).reshape(-1, W))
    ca = np.ascontiguousarray(c, dtype=np.float64)
    m = len(ca)
    ox = np.zeros((max(m, 1), W), dtype=np.uint64)
    oz = np.zeros((max(m, 1), W), dtype=np.uint64)
    oc = np.zeros(max(m, 1), dtype=np.float64)
    k = lib().orc_merge_records(n, GROUP_CODE[group], xa.ctypes.data_as(_u64p),
                                za.ctypes.data_as(_u64p), ca.ctypes.data_as(_f64p), m,
                                ox.ctypes.data_as(_u64p), oz.ctypes.data_as(_u64p),
                                oc.ctypes.data_as(_f64p))
    return {(_join(ox[i]), _join(oz[i])): float(oc[i]) for i in range(k)}


def int_less(n: int, a, b) -> bool:
    W = (n + 63) // 64
    return bool(lib().orc_int_less(n, _words(a[0], W), _words(a[1], W),
                                   _words(b[0], W), _words(b[1], W)))


class Oracle:
    """One propagation handle (a std::map of strings to FP64 coefficients)."""

    def __init__(self, n: int, group: str, lx: int = 0, perms=None):
        self.n, self.group, self.W = n, group, (n + 63) // 64
        if group == EXPLICIT:
            a, m = _perm_array(perms, n)
            self.h = lib().orc_create_group(n, a.ctypes.data, m)
        elif group == TORUS:
            self.h = lib().orc_create_torus(lx, n // lx if lx else 0)
        else:
            self.h = lib().orc_create(n, GROUP_CODE[group])
        if not self.h:
            raise ValueError(f"unsupported n={n}")

    def __del__(self):
        h, self.h = getattr(self, "h", None), None
        if h and _lib is not None:
            _lib.orc_destroy(h)

    def add(self, x: int, z: int, c: float):
        lib().orc_add_term(self.h, _words(x, self.W), _words(z, self.W), c)

    def merge(self):
        lib().orc_merge(self.h)

    def apply_gate(self, x: int, z: int, theta: float, eps: float, wmax: int):
        lib().orc_apply_gate(self.h, _words(x, self.W), _words(z, self.W), theta, eps, wmax)

    def damp(self, p: float):
        lib().orc_damp(self.h, p)

    def truncate(self, eps: float, wmax: int):
        lib().orc_truncate(self.h, eps, wmax)

    def expectation(self, bloch) -> float:
        return lib().orc_expectation(self.h, *map(float, bloch))

    def size(self) -> int:
        return lib().orc_size(self.h)

    def counters(self):
        p, m = ctypes.c_uint64(), ctypes.c_uint64()
        lib().orc_counters(self.h, ctypes.byref(p), ctypes.byref(m))
        return int(p.value), int(m.value)

    def export(self):
        """(x, z, c) arrays; x and z have shape (N, W) of uint64."""
        N = self.size()
        x = np.zeros((N, self.W), dtype=np.uint64)
        z = np.zeros((N, self.W), dtype=np.uint64)
        c = np.zeros(N, dtype=np.float64)
        if N:
            lib().orc_export(self.h, x.ctypes.data_as(_u64p), z.ctypes.data_as(_u64p),
                             c.ctypes.data_as(_f64p))
        return x, z, c

    def as_dict(self):
        x, z, c = self.export()
        return {(_join(x[i]), _join(z[i])): float(c[i]) for i in range(len(c))}


@dataclass
class OracleResult:
    expectation: float
    terms: dict
    propagated: int
    merged: int
    sizes: list          # set size after every sub-layer (after its truncation)
    peak: int            # largest set size seen after any gate
    wall: float
    sublayers_done: int
    rows: tuple | None = None    # export(): (x, z, c) in ascending integer order


def run_program(prog, group: str | None = None, max_sublayers: int | None = None,
                keep_terms: bool = True, time_budget: float | None = None,
                keep_rows: bool = False) -> OracleResult:
    """Algorithm 1 on the oracle.  ``max_sublayers``/``time_budget`` stop
    early (a bounded prefix, for timing samples)."""
    group = prog.group if group is None else group
    t0 = time.perf_counter()
    o = Oracle(prog.n, group, prog.meta.get("lx", 0), prog.meta.get("perms"))
    for (x, z, c) in prog.obs:
        o.add(x, z, c)
    o.merge()                                   # Algorithm 1, step 1
    sizes, peak, done = [], o.size(), 0
    for sub in reversed(prog.sublayers):        # step 2: l = L..1
        if max_sublayers is not None and done >= max_sublayers:
            break
        if time_budget is not None and time.perf_counter() - t0 > time_budget:
            break
        if sub.m != 1:
            raise ValueError("the oracle implements merge_every = 1")
        if sub.p > 0:
            o.damp(sub.p)
        for g in reversed(sub.gates):
            o.apply_gate(g.x, g.z, g.theta, sub.eps, sub.wmax)
            peak = max(peak, o.size())
        if getattr(sub, "merge", True):         # step 2b (deferred: Sec. IV's
            o.merge()                           # merge after a full Trotter layer)
        o.truncate(sub.eps, sub.wmax)
        sizes.append(o.size())
        done += 1
    e = o.expectation(prog.bloch)               # step 3
    prop, merged = o.counters()
    wall = time.perf_counter() - t0
    return OracleResult(e, o.as_dict() if keep_terms else {}, prop, merged, sizes,
                        peak, wall, done, o.export() if keep_rows else None)
