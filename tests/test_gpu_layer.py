"""Layer ops (pp_set_layer_ops): a sub-layer of 4..64 pairwise commuting
rotations applied bucket by bucket in two launches (strings bucketed by what
the rotations cannot change, every rotation of the sub-layer applied to a
bucket in LDS with the exact merge and truncation after each) gives bitwise
the results of the gate launches, on the one-instance program path, with
FP32 storage, with two key words, with the merge deferred to the end of a
Trotter layer (the op's output then carries gate-table entries), after
forced fallbacks to the gate launches, under store growth, and in the
batched form (which runs the gate copies); and the oracle's results by the
parity rules of tests/parity.py.  Algorithm 1 step 2a; Prop. 1."""
import pytest

from oracle import oracle as O
from paper_2512_12094_amd import workloads as W
from tests.parity import compare_expectation, compare_terms, compare_terms_f32

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
    yield dict(torch=torch, stream=stream, handle=int(stream.cuda_stream),
               alloc=_lib.TorchAllocator(0))
    _lib.pp_set_layer_ops(1)


def brickwork(n, steps, theta, eps):
    """Open chain of n qubits (two key words for n > 64), no symmetry: per
    step XX, YY, ZZ on the even bonds, then on the odd bonds (sub-layers of
    n/2 commuting rotations)."""
    subs = []
    for _ in range(steps):
        for kind in "XYZ":
            for parity in (0, 1):
                gates = [W.Gate(*W.two_site(kind, b, b + 1), theta)
                         for b in range(parity, n - 1, 2)]
                subs.append(W.SubLayer(gates, eps=eps))
    return W.Program(f"brick{n}", n, "none", W.sum_single(n, "Z"), subs, W.ZERO_STATE,
                     dict(eps=eps))


def prefix(prog, k):
    return W.Program(prog.name + f"[:{k}]", prog.n, prog.group, prog.obs,
                     prog.sublayers[len(prog.sublayers) - k:], prog.bloch, dict(prog.meta))


CASES = {
    "c1_z8": lambda: W.config1(),
    "c2_z32": lambda: prefix(W.config2(), 12),
    "ising_z12": lambda: W.tilted_ising_ring(12, 3, 0.25),
    "ising_z10_layer_merge": lambda: W.tilted_ising_ring(10, 3, 0.25, merge="layer"),
    "dn_12": lambda: W.xxz_ring(12, 2, 0.25, 1.3, eps=1e-6, group=W.GROUP_DN, name="dn12"),
    "torus_3x3": lambda: W.power_law_xxz_torus(3, 3, 1, 0.1, eps=1e-6),
    "plain_z10": lambda: W.xxz_ring(10, 2, 0.2, 1.0, eps=0.0, group="none", name="plain10"),
    "wide_z48": lambda: W.xxz_ring(48, 1, 0.2, 1.1, eps=1e-5, name="z48"),
    "two_words_n80": lambda: brickwork(80, 1, 0.3, 1e-6),
    "noise_z16": lambda: W.xxz_ring(16, 2, 0.3, 0.8, eps=1e-7, p=2e-3, name="z16p"),
}
ORACLE = ("c1_z8", "c2_z32", "ising_z12", "ising_z10_layer_merge", "torus_3x3", "two_words_n80")


def run(gpu, prog, mode, dtype="f64"):
    """The program on the one-instance path with layer ops in `mode`."""
    from paper_2512_12094_amd import _lib as L
    from paper_2512_12094_amd import driver
    L.pp_set_layer_ops(mode)
    try:
        dp = driver.DeviceProgram(prog)            # built under this mode
    finally:
        L.pp_set_layer_ops(1)
    L.pp_profile(None, 1)
    ps = driver.PauliSet.from_program(prog, None, gpu["handle"], gpu["alloc"], dtype)
    e = float(L.pp_batch_run([ps.h], [dp.h], gpu["handle"])[0])
    L.pp_profile(None, 0)
    prof = L.pp_profile_read(ps.h)
    prop, merged = ps.counters()
    terms = ps.as_dict()
    info = L.pp_program_info(dp.h)
    stats = L.pp_layer_stats(ps.h)
    ps.close()
    dp.close()
    return dict(e=e, terms=terms, prop=prop, merged=merged, prof=prof, info=info, stats=stats)


def same(a, b, what):
    assert a["terms"] == b["terms"], what            # bitwise, set and coefficients
    assert a["e"] == b["e"], (what, a["e"], b["e"])
    assert (a["prop"], a["merged"]) == (b["prop"], b["merged"]), what


@pytest.mark.parametrize("name", sorted(CASES))
def test_layer_ops_equal_gate_launches(gpu, name):
    prog = CASES[name]()
    print(f"[case] layer ops {name}", flush=True)
    on = run(gpu, prog, 1)
    off = run(gpu, prog, 0)
    forced = run(gpu, prog, 2)
    same(on, off, f"{name}: layer ops vs gate launches")
    same(forced, off, f"{name}: forced fallback vs gate launches")
    assert on["prof"]["layer_apply"][0] > 0, on["prof"]
    assert on["stats"]["layer_ops"] > 0, on["stats"]
    assert off["prof"]["layer_apply"][0] == 0
    assert forced["prof"]["gate"][0] > 0
    assert forced["stats"]["layer_ops"] == 0 and forced["stats"]["fallbacks"] > 0, forced["stats"]
    if name in ("c2_z32",):
        assert on["stats"]["fallbacks"] == 0, on["stats"]   # every sub-layer as one layer op
    if name in ORACLE:
        ref = O.run_program(prog)
        eps = prog.sublayers[0].eps
        compare_terms(on["terms"], ref.terms, eps, what=name)
        compare_expectation(on["e"], ref.expectation, ref.terms, what=name)
        assert (on["prop"], on["merged"]) == (ref.propagated, ref.merged)


def test_layer_ops_fp32(gpu):
    prog = CASES["c2_z32"]()
    print("[case] layer ops c2_z32 FP32", flush=True)
    on = run(gpu, prog, 1, "f32")
    off = run(gpu, prog, 0, "f32")
    same(on, off, "FP32 layer ops vs gate launches")
    ref = O.run_program(prog)
    compare_terms_f32(on["terms"], ref.terms, prog.sublayers[0].eps, what="c2 FP32")


def test_layer_ops_with_store_growth(gpu):
    """A Z_32 ring (theta 0.2, eps 1e-6, weight <= 12) whose set grows from
    32 strings to ~3x10^5 over 6 sub-layers: the store grows several times,
    some of them because a layer op's survivors did not fit."""
    full = W.xxz_ring(32, 5, 0.2, 1.5, eps=1e-6, wmax=12, obs=W.sum_ring_pairs(32, "X"),
                      name="ring32_scale")
    prog = prefix(full, 6)
    print("[case] layer ops with growth", flush=True)
    on = run(gpu, prog, 1)
    off = run(gpu, prog, 0)
    same(on, off, "growth: layer ops vs gate launches")
    assert on["prof"]["grow"][0] > 0


@pytest.mark.parametrize("mode", [1, 2])
def test_batched_form_runs_layer_ops(gpu, mode):
    """Programs with layer ops in the batched form (several instances,
    uneven n): the batched steps run the layer ops (mode 1) or, when every
    layer op reports a failure (mode 2), send the instances to the gate
    copies on the device; either way every instance equals its
    one-instance run bitwise."""
    from paper_2512_12094_amd import _lib as L
    from paper_2512_12094_amd import driver
    progs = [CASES[k]() for k in ("c1_z8", "dn_12", "noise_z16", "c2_z32", "two_words_n80")]
    print(f"[case] batched programs with layer ops, mode {mode}", flush=True)
    L.pp_set_layer_ops(mode)
    try:
        dprogs = [driver.DeviceProgram(p) for p in progs]
    finally:
        L.pp_set_layer_ops(1)
    sets = [driver.PauliSet.from_program(p, None, gpu["handle"], gpu["alloc"]) for p in progs]
    e = L.pp_batch_run([s.h for s in sets], [d.h for d in dprogs], gpu["handle"])
    for p, s, d, ei in zip(progs, sets, dprogs, e):
        solo = run(gpu, p, 1)
        assert s.as_dict() == solo["terms"], p.name
        assert float(ei) == solo["e"], p.name
        assert s.counters() == (solo["prop"], solo["merged"]), p.name
        st = L.pp_layer_stats(s.h)
        if mode == 1:
            assert st["layer_ops"] > 0, (p.name, st)
        else:
            assert st["layer_ops"] == 0 and st["fallbacks"] > 0, (p.name, st)
        s.close()
        d.close()
