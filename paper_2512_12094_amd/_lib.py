"""ctypes binding of libpp.so (include/pp.h), argument marshalling only.

Every function here has the name of the C entry point it calls and does
nothing but convert Python/numpy arguments, call it, and raise on a negative
status.  All propagation work runs in the HIP kernels of libpp.so; there is
no CPU fallback: loading fails loudly when the library or a GPU is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpp.so")

PP_GROUP = {"none": 0, "Zn": 1, "Sn": 2, "Dn": 3, "T2": 4, "G": 5}
PP_F64 = 0
PP_F32_COMPENSATED = 1
DTYPES = {"f64": PP_F64, "f32": PP_F32_COMPENSATED}
ERRORS = {-1: "PP_EINVAL", -2: "PP_ENOTSYM", -3: "PP_ENOMEM", -4: "PP_ECAPACITY",
          -5: "PP_EDEVICE"}

_u64p = ctypes.POINTER(ctypes.c_uint64)
_f64p = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class PPAllocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p)]


class PPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    """Loads libpp.so; raises if it is missing (never falls back)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(LIB_PATH)
    L.pp_last_error.restype = ctypes.c_char_p
    L.pp_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                            _u64p, _u64p, _f64p, ctypes.c_size_t, _vp,
                            ctypes.POINTER(PPAllocator)]
    L.pp_create_group.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, _vp, ctypes.c_size_t,
                                  ctypes.c_int, _u64p, _u64p, _f64p, ctypes.c_size_t, _vp,
                                  ctypes.POINTER(PPAllocator)]
    L.pp_create_torus.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  _u64p, _u64p, _f64p, ctypes.c_size_t, _vp,
                                  ctypes.POINTER(PPAllocator)]
    L.pp_apply_layer.argtypes = [_vp, _u64p, _u64p, _f64p, ctypes.c_size_t, ctypes.c_int,
                                 ctypes.c_double, ctypes.c_int]
    L.pp_merge_canonicalize.argtypes = [_vp]
    L.pp_truncate.argtypes = [_vp, ctypes.c_double, ctypes.c_int, ctypes.c_double]
    L.pp_expectation.argtypes = [_vp, _f64p, _f64p]
    L.pp_expectation_noalloc.argtypes = [_vp, _f64p, _f64p]
    L.pp_num_terms.argtypes = [_vp, ctypes.POINTER(ctypes.c_size_t)]
    L.pp_peak_terms.argtypes = [_vp, ctypes.POINTER(ctypes.c_size_t)]
    L.pp_store_bytes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_size_t,
                                 ctypes.POINTER(ctypes.c_size_t)]
    L.pp_export_terms.argtypes = [_vp, _u64p, _u64p, _f64p, ctypes.c_size_t,
                                  ctypes.POINTER(ctypes.c_size_t)]
    L.pp_counters.argtypes = [_vp, _u64p]
    L.pp_set_max_terms.argtypes = [_vp, ctypes.c_size_t]
    L.pp_work_counters.argtypes = [_vp, _u64p]
    L.pp_merge_stats.argtypes = [_vp, _u64p]
    L.pp_profile.argtypes = [_vp, ctypes.c_int]
    L.pp_profile_read.argtypes = [_vp, _u64p, _f64p]
    L.pp_destroy.argtypes = [_vp]
    L.pp_destroy.restype = None
    L.pp_program_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_size_t,
                                    ctypes.POINTER(ctypes.c_size_t), _u64p, _u64p, _f64p,
                                    _f64p, ctypes.POINTER(ctypes.c_int), _f64p, _f64p,
                                    ctypes.POINTER(ctypes.c_int)]
    L.pp_program_destroy.argtypes = [_vp]
    L.pp_program_destroy.restype = None
    L.pp_program_info.argtypes = [_vp, ctypes.POINTER(ctypes.c_uint64)]
    L.pp_batch_run.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.c_size_t, _vp,
                               _f64p]
    L.pp_batch_step.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.c_size_t, _vp,
                                ctypes.c_int, ctypes.POINTER(ctypes.c_int), _f64p]
    L.pp_set_tuning.argtypes = [ctypes.c_int] * 5
    L.pp_set_gate_fusion.argtypes = [ctypes.c_int, ctypes.c_int]
    L.pp_set_layer_ops.argtypes = [ctypes.c_int]
    L.pp_layer_stats.argtypes = [_vp, _u64p]
    L.pp_set_layer_tuning.argtypes = [ctypes.c_int, ctypes.c_int]
    L.pp_get_layer_tuning.argtypes = [ctypes.POINTER(ctypes.c_int)]
    L.pp_get_tuning.argtypes = [ctypes.POINTER(ctypes.c_int)]
    L.pp_set_merge_tuning.argtypes = [ctypes.c_int, ctypes.c_int]
    L.pp_get_merge_tuning.argtypes = [ctypes.POINTER(ctypes.c_int)]
    _lib = L
    return L


def _check(rc):
    if rc != 0:
        raise PPError(rc, lib().pp_last_error().decode())


def _u64(a):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return a, a.ctypes.data_as(_u64p)


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_f64p)


# ---------------------------------------------------------------------------
# device memory and streams come from PyTorch
# ---------------------------------------------------------------------------
class TorchAllocator:
    """pp_allocator backed by PyTorch's caching allocator."""

    def __init__(self, device: int = 0):
        import torch
        self.torch = torch
        self.device = device

        def _alloc(nbytes, stream, ctx):
            try:
                return int(torch.cuda.caching_allocator_alloc(int(nbytes), self.device,
                                                              int(stream or 0)))
            except Exception:   # out of memory: the library reports PP_ENOMEM
                return None

        def _free(ptr, stream, ctx):
            if ptr:
                torch.cuda.caching_allocator_delete(int(ptr))

        self._alloc, self._free = ALLOC_FN(_alloc), FREE_FN(_free)
        self.struct = PPAllocator(self._alloc, self._free, None)


def current_stream_handle():
    import torch
    return int(torch.cuda.current_stream().cuda_stream)


# ---------------------------------------------------------------------------
# entry points (same names as include/pp.h)
# ---------------------------------------------------------------------------
def pp_create(n, group, obs_x, obs_z, obs_coef, stream=0, allocator=None, dtype="f64"):
    """obs_x/obs_z: (rows, W) uint64 arrays; obs_coef: (rows,) float64;
    dtype "f64" (PP_F64) or "f32" (PP_F32_COMPENSATED)."""
    W = (n + 63) // 64
    x, xp = _u64(np.asarray(obs_x, dtype=np.uint64).reshape(-1, W))
    z, zp = _u64(np.asarray(obs_z, dtype=np.uint64).reshape(-1, W))
    c, cp = _f64(obs_coef)
    h = _vp()
    al = ctypes.byref(allocator.struct) if allocator is not None else None
    _check(lib().pp_create(ctypes.byref(h), n, PP_GROUP.get(group, group),
                           DTYPES.get(dtype, dtype), xp, zp, cp, len(c), _vp(stream or None), al))
    return h


def pp_create_group(n, perms, obs_x, obs_z, obs_coef, stream=0, allocator=None, dtype="f64"):
    """pp_create for the group whose elements are the rows of perms (each a
    list of n qubit indices: qubit q of g.s carries qubit perms[g][q] of s)."""
    W = (n + 63) // 64
    p = np.ascontiguousarray(np.asarray(perms, dtype=np.uint8).reshape(-1, n))
    x, xp = _u64(np.asarray(obs_x, dtype=np.uint64).reshape(-1, W))
    z, zp = _u64(np.asarray(obs_z, dtype=np.uint64).reshape(-1, W))
    c, cp = _f64(obs_coef)
    h = _vp()
    al = ctypes.byref(allocator.struct) if allocator is not None else None
    _check(lib().pp_create_group(ctypes.byref(h), n, p.ctypes.data_as(_vp), len(p),
                                 DTYPES.get(dtype, dtype), xp, zp, cp, len(c),
                                 _vp(stream or None), al))
    return h


def pp_create_torus(lx, ly, obs_x, obs_z, obs_coef, stream=0, allocator=None, dtype="f64"):
    """pp_create for the translations of an lx x ly torus (n = lx * ly)."""
    n = lx * ly
    W = (n + 63) // 64
    x, xp = _u64(np.asarray(obs_x, dtype=np.uint64).reshape(-1, W))
    z, zp = _u64(np.asarray(obs_z, dtype=np.uint64).reshape(-1, W))
    c, cp = _f64(obs_coef)
    h = _vp()
    al = ctypes.byref(allocator.struct) if allocator is not None else None
    _check(lib().pp_create_torus(ctypes.byref(h), lx, ly, DTYPES.get(dtype, dtype), xp, zp, cp,
                                 len(c), _vp(stream or None), al))
    return h


def pp_apply_layer(h, gate_x, gate_z, theta, W, merge_every=1, inner_eps=0.0,
                   inner_max_weight=-1):
    x, xp = _u64(np.asarray(gate_x, dtype=np.uint64).reshape(-1, W))
    z, zp = _u64(np.asarray(gate_z, dtype=np.uint64).reshape(-1, W))
    t, tp = _f64(theta)
    _check(lib().pp_apply_layer(h, xp, zp, tp, len(t), merge_every, inner_eps,
                                inner_max_weight))


def pp_merge_canonicalize(h):
    _check(lib().pp_merge_canonicalize(h))


def pp_truncate(h, eps=0.0, max_weight=-1, depol_p=0.0):
    _check(lib().pp_truncate(h, eps, max_weight, depol_p))


def pp_expectation(h, bloch) -> float:
    b, bp = _f64(np.asarray(bloch, dtype=np.float64))
    out = ctypes.c_double()
    _check(lib().pp_expectation(h, bp, ctypes.byref(out)))
    return out.value


def pp_expectation_noalloc(h, bloch) -> float:
    b, bp = _f64(np.asarray(bloch, dtype=np.float64))
    out = ctypes.c_double()
    _check(lib().pp_expectation_noalloc(h, bp, ctypes.byref(out)))
    return out.value


def pp_store_bytes(n, group, cap, dtype="f64") -> int:
    out = ctypes.c_size_t()
    _check(lib().pp_store_bytes(int(n), PP_GROUP[group] if isinstance(group, str) else int(group),
                                DTYPES[dtype] if isinstance(dtype, str) else int(dtype),
                                int(cap), ctypes.byref(out)))
    return int(out.value)


def pp_peak_terms(h) -> int:
    out = ctypes.c_size_t()
    _check(lib().pp_peak_terms(h, ctypes.byref(out)))
    return int(out.value)


def pp_num_terms(h) -> int:
    out = ctypes.c_size_t()
    _check(lib().pp_num_terms(h, ctypes.byref(out)))
    return out.value


def pp_export_terms(h, W):
    n = pp_num_terms(h)
    x = np.zeros((max(n, 1), W), dtype=np.uint64)
    z = np.zeros((max(n, 1), W), dtype=np.uint64)
    c = np.zeros(max(n, 1), dtype=np.float64)
    got = ctypes.c_size_t()
    _check(lib().pp_export_terms(h, x.ctypes.data_as(_u64p), z.ctypes.data_as(_u64p),
                                 c.ctypes.data_as(_f64p), n, ctypes.byref(got)))
    k = got.value
    return x[:k], z[:k], c[:k]


def pp_counters(h):
    out = (ctypes.c_uint64 * 2)()
    _check(lib().pp_counters(h, out))
    return int(out[0]), int(out[1])


KERNELS = ["gate", "merge_narrow", "merge_wide1", "merge_wide2", "merge_collect", "compact",
           "scan", "grow", "part_hist", "part_scan", "part_scatter", "part_agg",
           "layer_scatter", "layer_apply"]


def pp_work_counters(h):
    out = (ctypes.c_uint64 * 8)()
    _check(lib().pp_work_counters(h, out))
    keys = ["propagated", "merged", "anticommuting", "appended", "merge_in", "merge_out",
            "gate_key_reads", "gate_coef_rw"]
    return {k: int(v) for k, v in zip(keys, out)}


def pp_merge_stats(h):
    out = (ctypes.c_uint64 * 4)()
    _check(lib().pp_merge_stats(h, out))
    keys = ["partitioned_merges", "split_buckets", "selector_buckets", "global_keys"]
    return {k: int(v) for k, v in zip(keys, out)}


def pp_profile(h, every=1):
    """every: bracket every `every`-th launch per kernel kind (0 = off)."""
    _check(lib().pp_profile(h, int(every)))


def pp_profile_read(h):
    n = (ctypes.c_uint64 * len(KERNELS))()
    ms = (ctypes.c_double * len(KERNELS))()
    _check(lib().pp_profile_read(h, n, ms))
    return {k: (int(n[i]), float(ms[i])) for i, k in enumerate(KERNELS)}


def pp_set_max_terms(h, max_terms):
    _check(lib().pp_set_max_terms(h, max_terms))


def pp_destroy(h):
    if h:
        lib().pp_destroy(h)


def pp_program_create(n, sub_start, gate_x, gate_z, theta, eps, max_weight, depol_p, bloch,
                      merge_after=None):
    W = (n + 63) // 64
    ss = np.ascontiguousarray(sub_start, dtype=np.uint64)
    x, xp = _u64(np.asarray(gate_x, dtype=np.uint64).reshape(-1, W))
    z, zp = _u64(np.asarray(gate_z, dtype=np.uint64).reshape(-1, W))
    t, tp = _f64(theta)
    e, ep = _f64(eps)
    w = np.ascontiguousarray(max_weight, dtype=np.int32)
    p, pq = _f64(depol_p)
    b, bp = _f64(np.asarray(bloch, dtype=np.float64))
    mp = None
    if merge_after is not None:
        m = np.ascontiguousarray(merge_after, dtype=np.int32)
        mp = m.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    h = _vp()
    _check(lib().pp_program_create(
        ctypes.byref(h), n, len(ss) - 1, ss.ctypes.data_as(ctypes.POINTER(ctypes.c_size_t)),
        xp, zp, tp, ep, w.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), pq, bp, mp))
    return h


def pp_program_info(h):
    out = (ctypes.c_uint64 * 4)()
    _check(lib().pp_program_info(h, out))
    return dict(ops=int(out[0]), gate_launches=int(out[1]), gates=int(out[2]),
                layer_ops=int(out[3]))


def pp_program_destroy(h):
    if h:
        lib().pp_program_destroy(h)


def pp_batch_run(states, programs, stream):
    n = len(states)
    S = (_vp * n)(*[s.value if isinstance(s, _vp) else s for s in states])
    P = (_vp * n)(*[p.value if isinstance(p, _vp) else p for p in programs])
    out = np.zeros(n, dtype=np.float64)
    _check(lib().pp_batch_run(S, P, n, _vp(stream), out.ctypes.data_as(_f64p)))
    return out


def pp_batch_step(states, programs, stream, max_steps):
    n = len(states)
    S = (_vp * n)(*[s.value if isinstance(s, _vp) else s for s in states])
    P = (_vp * n)(*[p.value if isinstance(p, _vp) else p for p in programs])
    done = (ctypes.c_int * n)()
    out = np.zeros(n, dtype=np.float64)
    _check(lib().pp_batch_step(S, P, n, _vp(stream), max_steps, done,
                               out.ctypes.data_as(_f64p)))
    return np.array(list(done), dtype=np.int32), out


TUNING_KEYS = ["gate_items", "stream_items", "max_blocks", "graph_steps", "gates_per_step"]


def pp_set_tuning(gate_items=0, stream_items=0, max_blocks=0, graph_steps=0, gates_per_step=0):
    _check(lib().pp_set_tuning(gate_items, stream_items, max_blocks, graph_steps,
                               gates_per_step))


def pp_set_gate_fusion(max_rotations, lanes=0):
    """Rotations one gate launch may apply (0 or 1: no fusion; 2 or 3), and
    whether smaller sets run fused ops with one lane per group member."""
    _check(lib().pp_set_gate_fusion(int(max_rotations), int(lanes)))


def pp_set_layer_ops(mode):
    """Layer ops for programs created afterwards: 0 off, 1 on, 2 on with
    every layer op falling back to its gate launches."""
    _check(lib().pp_set_layer_ops(int(mode)))


def pp_set_layer_tuning(bucket_log2=0, block=0):
    """Layer ops: log2 strings per bucket (4..10; 0 keeps) and threads per
    bucket block (256 or 512; 0 keeps)."""
    _check(lib().pp_set_layer_tuning(int(bucket_log2), int(block)))


def pp_layer_stats(h):
    """Layer ops completed, runs that overflowed a bucket, ops replaced by
    their gate launches, and whether the handle runs gate launches only."""
    out = np.zeros(4, dtype=np.uint64)
    _check(lib().pp_layer_stats(h, out.ctypes.data_as(_u64p)))
    return dict(layer_ops=int(out[0]), overflow_runs=int(out[1]), fallbacks=int(out[2]),
                gates_only=bool(out[3]))


def pp_get_layer_tuning():
    out = (ctypes.c_int * 2)()
    _check(lib().pp_get_layer_tuning(out))
    return dict(bucket_log2=out[0], block=out[1])


def pp_get_tuning():
    out = (ctypes.c_int * 5)()
    _check(lib().pp_get_tuning(out))
    return dict(zip(TUNING_KEYS, list(out)))


def pp_set_merge_tuning(bucket_log2=0, agg_blocks=0):
    _check(lib().pp_set_merge_tuning(int(bucket_log2), int(agg_blocks)))


def pp_get_merge_tuning():
    out = (ctypes.c_int * 2)()
    _check(lib().pp_get_merge_tuning(out))
    return dict(bucket_log2=int(out[0]), agg_blocks=int(out[1]))
