"""Algorithm 1 of arXiv:2512.12094 on the GPU, through the C ABI only.

``propagate`` walks a ``workloads.Program`` exactly as the paper's
Algorithm 1 does: merge the observable by orbit representative (step 1),
then for every sub-layer in Heisenberg order damp, apply its rotations
(each followed by the exact merge and the truncation), merge by
representative (step 2b) and truncate; finally the expectation in the
symmetric product state (step 3).  Each of those steps is one call into
libpp.so; this module only prepares arrays.

``program_arrays``/``BatchRunner`` describe whole programs for the batched
form (pp_program_create / pp_batch_run).
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import _lib as L
from .workloads import Program, n_words


def _rows(ints, W):
    out = np.zeros((len(ints), W), dtype=np.uint64)
    for r, v in enumerate(ints):
        for w in range(W):
            out[r, w] = (v >> (64 * w)) & 0xFFFFFFFFFFFFFFFF
    return out


@dataclass
class LayerArrays:
    gx: np.ndarray
    gz: np.ndarray
    theta: np.ndarray
    eps: float
    wmax: int
    p: float
    merge: bool = True


def heisenberg_layers(prog: Program):
    """Sub-layers in Heisenberg order, each with its gates in the order they
    are applied (the time-ordered lists walked backwards)."""
    cache = prog.meta.get("_heis")
    if cache is not None:
        return cache
    W = n_words(prog.n)
    out = []
    for sub in reversed(prog.sublayers):
        if sub.m != 1:
            raise ValueError("only merge_every = 1 is supported")
        gates = list(reversed(sub.gates))
        out.append(LayerArrays(_rows([g.x for g in gates], W), _rows([g.z for g in gates], W),
                               np.array([g.theta for g in gates], dtype=np.float64),
                               float(sub.eps), int(sub.wmax), float(sub.p),
                               bool(getattr(sub, "merge", True))))
    prog.meta["_heis"] = out
    return out


def observable_arrays(prog: Program):
    W = n_words(prog.n)
    return (_rows([o[0] for o in prog.obs], W), _rows([o[1] for o in prog.obs], W),
            np.array([o[2] for o in prog.obs], dtype=np.float64))


@dataclass
class GpuResult:
    expectation: float
    terms: dict
    propagated: int
    merged: int
    sizes: list
    wall: float
    extra: dict = field(default_factory=dict)


class PauliSet:
    """A handle (pp_state) with the observable loaded and merged."""

    def __init__(self, n: int, group: str, obs_x, obs_z, obs_c, stream: int = 0,
                 allocator=None, dtype: str = "f64", lx: int = 0, perms=None):
        self.n, self.group, self.W, self.dtype = n, group, n_words(n), dtype
        if group == "G":
            self.h = L.pp_create_group(n, perms, obs_x, obs_z, obs_c, stream, allocator, dtype)
        elif group == "T2":
            self.h = L.pp_create_torus(lx, n // lx, obs_x, obs_z, obs_c, stream, allocator,
                                       dtype)
        else:
            self.h = L.pp_create(n, group, obs_x, obs_z, obs_c, stream, allocator, dtype)
        self._allocator = allocator

    @classmethod
    def from_program(cls, prog: Program, group: str | None = None, stream: int = 0,
                     allocator=None, dtype: str = "f64"):
        x, z, c = observable_arrays(prog)
        return cls(prog.n, prog.group if group is None else group, x, z, c, stream, allocator,
                   dtype, prog.meta.get("lx", 0), prog.meta.get("perms"))

    def apply_layer(self, la: LayerArrays):
        L.pp_apply_layer(self.h, la.gx, la.gz, la.theta, self.W, 1, la.eps, la.wmax)

    def merge(self):
        L.pp_merge_canonicalize(self.h)

    def truncate(self, eps=0.0, wmax=-1, p=0.0):
        L.pp_truncate(self.h, eps, wmax, p)

    def expectation(self, bloch) -> float:
        return L.pp_expectation(self.h, bloch)

    def num_terms(self) -> int:
        return L.pp_num_terms(self.h)

    def counters(self):
        return L.pp_counters(self.h)

    def export(self):
        return L.pp_export_terms(self.h, self.W)

    def as_dict(self):
        x, z, c = self.export()
        out = {}
        for i in range(len(c)):
            xi = sum(int(x[i, w]) << (64 * w) for w in range(self.W))
            zi = sum(int(z[i, w]) << (64 * w) for w in range(self.W))
            out[(xi, zi)] = float(c[i])
        return out

    def close(self):
        if self.h:
            L.pp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_layers(ps: PauliSet, layers, record_sizes=False):
    sizes = []
    for la in layers:
        if la.p > 0:
            ps.truncate(0.0, -1, la.p)
        ps.apply_layer(la)
        if la.merge:
            ps.merge()
        if la.eps > 0 or la.wmax >= 0:
            ps.truncate(la.eps, la.wmax, 0.0)
        if record_sizes:
            sizes.append(ps.num_terms())
    return sizes


def propagate(prog: Program, group: str | None = None, keep_terms: bool = True,
              stream: int = 0, allocator=None, record_sizes: bool = False,
              max_sublayers: int | None = None, dtype: str = "f64") -> GpuResult:
    """Algorithm 1 through the C ABI; returns the expectation (and the final
    representative set when keep_terms)."""
    layers = heisenberg_layers(prog)
    if max_sublayers is not None:
        layers = layers[:max_sublayers]
    t0 = time.perf_counter()
    ps = PauliSet.from_program(prog, group, stream, allocator, dtype)
    sizes = run_layers(ps, layers, record_sizes)
    e = ps.expectation(prog.bloch)
    wall = time.perf_counter() - t0
    prop, merged = ps.counters()
    terms = ps.as_dict() if keep_terms else {}
    ps.close()
    return GpuResult(e, terms, prop, merged, sizes, wall)


# ---------------------------------------------------------------------------
# batched form
# ---------------------------------------------------------------------------
def program_arrays(prog: Program):
    layers = heisenberg_layers(prog)
    W = n_words(prog.n)
    starts = [0]
    for la in layers:
        starts.append(starts[-1] + len(la.theta))
    gx = np.concatenate([la.gx for la in layers]) if layers else np.zeros((0, W), np.uint64)
    gz = np.concatenate([la.gz for la in layers]) if layers else np.zeros((0, W), np.uint64)
    th = np.concatenate([la.theta for la in layers]) if layers else np.zeros(0)
    eps = np.array([la.eps for la in layers], dtype=np.float64)
    wmax = np.array([la.wmax for la in layers], dtype=np.int32)
    p = np.array([la.p for la in layers], dtype=np.float64)
    merge = np.array([1 if la.merge else 0 for la in layers], dtype=np.int32)
    return starts, gx, gz, th, eps, wmax, p, merge


class DeviceProgram:
    """A whole propagation uploaded once (pp_program_create)."""

    def __init__(self, prog: Program):
        self.prog = prog
        starts, gx, gz, th, eps, wmax, p, merge = program_arrays(prog)
        self.h = L.pp_program_create(prog.n, starts, gx, gz, th, eps, wmax, p, prog.bloch,
                                     merge_after=merge)

    def close(self):
        if self.h:
            L.pp_program_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def device_program(prog: Program) -> "DeviceProgram":
    """The program uploaded once and cached on the Program object."""
    dp = prog.meta.get("_dprog")
    if dp is None or dp.h is None:
        dp = DeviceProgram(prog)
        prog.meta["_dprog"] = dp
    return dp


def propagate_program(prog: Program, group: str | None = None, stream: int = 0,
                      allocator=None, keep_terms: bool = False, dtype: str = "f64") -> GpuResult:
    """Algorithm 1 as one device program (pp_program + pp_batch_run with one
    instance): all sub-layers are queued ahead and the host only checks the
    device status between sub-layers."""
    dp = device_program(prog)
    t0 = time.perf_counter()
    ps = PauliSet.from_program(prog, group, stream, allocator, dtype)
    e = float(L.pp_batch_run([ps.h], [dp.h], stream)[0])
    wall = time.perf_counter() - t0
    prop, merged = ps.counters()
    terms = ps.as_dict() if keep_terms else {}
    ps.close()
    return GpuResult(e, terms, prop, merged, [], wall)


def batch_propagate(progs, stream: int, allocator=None, group=None, dtype: str = "f64"):
    """All programs in one batched run; returns (expectations, handles)."""
    sets = [PauliSet.from_program(p, group, stream, allocator, dtype) for p in progs]
    dprogs = [DeviceProgram(p) for p in progs]
    t0 = time.perf_counter()
    e = L.pp_batch_run([s.h for s in sets], [d.h for d in dprogs], stream)
    wall = time.perf_counter() - t0
    return e, sets, dprogs, wall
