"""Gate fusion (pp_set_gate_fusion): a launch that applies two or three
commuting, independent rotations of a sub-layer, each with its own exact
merge and truncation, gives bitwise the results of one launch per gate (same
arithmetic in the same order), on every path (per-call layers, the
one-instance program, the batched form, FP32 storage, store growth), and the
oracle's results by the parity rules of tests/parity.py; the gate launch
count drops by the group size.  Programs here are built with layer ops off
(tests/test_gpu_layer.py covers those)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2512_12094_amd import workloads as W
from tests.parity import compare_expectation, compare_terms

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
    _lib.pp_set_layer_ops(0)             # programs run their gate launches here
    yield dict(torch=torch, stream=stream, handle=int(stream.cuda_stream),
               alloc=_lib.TorchAllocator(0))
    _lib.pp_set_gate_fusion(3, 0)
    _lib.pp_set_layer_ops(1)


def prefix(prog, k):
    return W.Program(prog.name + f"[:{k}]", prog.n, prog.group, prog.obs,
                     prog.sublayers[len(prog.sublayers) - k:], prog.bloch, dict(prog.meta))


def ising(n, steps, dt, eps, wmax, gx=1.4, gz=0.9045):
    """Tilted-field Ising ring with truncation (ZZ bonds, Z field, X field)."""
    kw = dict(eps=eps, wmax=wmax)
    subs = []
    for _ in range(steps):
        subs += [W.ring_sublayer(n, "Z", 2 * dt, **kw), W.field_sublayer(n, "Z", 2 * gz * dt, **kw),
                 W.field_sublayer(n, "X", 2 * gx * dt, **kw)]
    return W.Program(f"ising{n}", n, W.GROUP_ZN, W.sum_single(n, "Z"), subs, W.ZERO_STATE,
                     dict(eps=eps, wmax=wmax))


CASES = {
    "c1_z8": lambda: W.config1(),
    "c2_z32": lambda: prefix(W.config2(), 12),
    "c3_s20": lambda: prefix(W.config3(), 2),           # grows the store
    "heis_s10_noise": lambda: W.heisenberg_all_to_all(10, 2, 0.1, eps=1e-5, p=1e-3,
                                                      name="s10"),
    "ising_z12_wmax": lambda: ising(12, 3, 0.1, 1e-5, 5),
    "plain_z10": lambda: W.xxz_ring(10, 2, 0.2, 1.0, eps=0.0, group="none", name="plain10"),
    "dn_12": lambda: W.xxz_ring(12, 2, 0.25, 1.3, eps=1e-6, group=W.GROUP_DN, name="dn12"),
    "torus_4x4": lambda: W.power_law_xxz_torus(4, 4, 1, 0.1, eps=1e-4),
    "wide_z48": lambda: W.xxz_ring(48, 1, 0.2, 1.1, eps=1e-5, name="z48"),
    "two_words_n80": lambda: W.xxz_ring(80, 1, 0.2, 1.1, eps=1e-5, group="none", name="n80"),
}


def run_program(gpu, prog, fuse, dtype="f64", lanes=0):
    from paper_2512_12094_amd import _lib as L, driver
    L.pp_set_gate_fusion(fuse, lanes)
    prog.meta.pop("_dprog", None)          # the program is rebuilt with the setting
    res = driver.propagate_program(prog, stream=gpu["handle"], allocator=gpu["alloc"],
                                   keep_terms=True, dtype=dtype)
    prog.meta.pop("_dprog", None)
    return res


def same(a, b, what):
    assert a.expectation == b.expectation, (what, a.expectation, b.expectation)
    assert (a.propagated, a.merged) == (b.propagated, b.merged), what
    assert a.terms == b.terms, what


@pytest.mark.parametrize("which", list(CASES))
def test_fused_program_equals_unfused_and_oracle(gpu, which):
    prog = CASES[which]()
    print(f"[case] fusion program {which}", flush=True)
    plain = run_program(gpu, prog, 1)
    for k in (2, 3):
        for lanes in (0, 1):                   # one thread per term, one lane per member
            fused = run_program(gpu, prog, k, lanes=lanes)
            same(fused, plain, f"{which} fused {k} lanes {lanes}")
    ref = O.run_program(prog)
    compare_terms(fused.terms, ref.terms, prog.meta.get("eps", 0.0), what=which)
    compare_expectation(fused.expectation, ref.expectation, ref.terms, what=which)
    assert (fused.propagated, fused.merged) == (ref.propagated, ref.merged), which


@pytest.mark.parametrize("which", ["c1_z8", "heis_s10_noise", "ising_z12_wmax", "dn_12"])
def test_fused_layers_equal_unfused(gpu, which):
    """The per-call path (pp_apply_layer per sub-layer)."""
    from paper_2512_12094_amd import _lib as L, driver
    prog = CASES[which]()
    print(f"[case] fusion layers {which}", flush=True)
    out = []
    for fuse, lanes in ((3, 1), (2, 1), (3, 0), (1, 1)):
        L.pp_set_gate_fusion(fuse, lanes)
        out.append(driver.propagate(prog, stream=gpu["handle"], allocator=gpu["alloc"]))
    for o in out[:3]:
        same(o, out[3], which)


def test_fused_f32_equals_unfused_f32(gpu):
    prog = prefix(W.config2(), 12)
    print("[case] fusion f32", flush=True)
    plain = run_program(gpu, prog, 1, "f32")
    for k in (2, 3):
        for lanes in (0, 1):
            same(run_program(gpu, prog, k, "f32", lanes), plain, f"f32 fused {k} lanes {lanes}")


def test_fused_batch_equals_unfused(gpu):
    """Batched form: instances at fused and one-gate ops in the same launch."""
    from paper_2512_12094_amd import _lib as L, driver
    rng = np.random.default_rng(5)
    progs = []
    for k in range(6):
        n = int(rng.choice([8, 12, 16, 40, 70]))
        progs.append(W.xxz_ring(n, int(rng.integers(1, 3)), float(rng.uniform(0.05, 0.3)),
                                float(rng.uniform(0.5, 2)), eps=1e-6, name=f"f{k}_n{n}"))
    progs.append(ising(9, 2, 0.1, 1e-6, -1))
    progs.append(W.heisenberg_all_to_all(9, 1, 0.1, eps=1e-5, name="fs9"))
    print("[case] fusion batch", [p.n for p in progs], flush=True)
    results = []
    for fuse in (3, 1, 2):
        L.pp_set_gate_fusion(fuse)
        e, sets, dprogs, _ = driver.batch_propagate(progs, gpu["handle"], gpu["alloc"])
        results.append((list(e), [s.as_dict() for s in sets], [s.counters() for s in sets]))
        for s in sets:
            s.close()
        for d in dprogs:
            d.close()
    assert results[0] == results[1]
    assert results[2] == results[1]
    for p, ei, terms, cnt in zip(progs, *results[0]):
        ref = O.run_program(p)
        compare_expectation(ei, ref.expectation, ref.terms, what=p.name)
        assert cnt == (ref.propagated, ref.merged), p.name


def test_fusion_divides_gate_launches(gpu):
    """All gates of a ring sub-layer commute and any three neighbouring bonds
    are independent: n gates take ceil(n / k) launches."""
    from paper_2512_12094_amd import _lib as L, driver
    prog = W.xxz_ring(16, 1, 0.2, 1.0, eps=1e-6, name="z16")
    counts = []
    for fuse in (3, 2, 1):
        L.pp_set_gate_fusion(fuse)
        ps = driver.PauliSet.from_program(prog, None, gpu["handle"], gpu["alloc"])
        L.pp_profile(ps.h, 1)
        for la in driver.heisenberg_layers(prog):
            ps.apply_layer(la)
        counts.append(L.pp_profile_read(ps.h)["gate"][0])
        ps.close()
    assert counts == [3 * 6, 3 * 8, 3 * 16], counts


def test_fusion_switch_validates():
    from paper_2512_12094_amd import _lib as L
    for bad in ((-1, 1), (4, 1), (3, 2)):
        with pytest.raises(L.PPError):
            L.pp_set_gate_fusion(*bad)
    L.pp_set_gate_fusion(3, 0)


def test_gate_unit_counters_and_program_info(gpu):
    """Without fusion every launch reads the keys of the live terms entering
    it and rewrites the anticommuting ones: the byte-model counters equal
    the per-gate counters.  With fusion a launch reads each key once for two
    rotations: fewer reads, the same work units (propagated, merged)."""
    from paper_2512_12094_amd import _lib as L, driver
    prog = prefix(W.config2(), 6)
    wcs = []
    for fuse in (1, 3):
        L.pp_set_gate_fusion(fuse)
        prog.meta.pop("_dprog", None)
        dp = driver.device_program(prog)
        info = L.pp_program_info(dp.h)
        assert info["gates"] == prog.n_gates
        per_sub = -(-prog.n // fuse)                 # ring sub-layers group up
        assert info["gate_launches"] == per_sub * len(prog.sublayers)
        ps = driver.PauliSet.from_program(prog, None, gpu["handle"], gpu["alloc"])
        L.pp_batch_run([ps.h], [dp.h], gpu["handle"])
        wcs.append(L.pp_work_counters(ps.h))
        ps.close()
        prog.meta.pop("_dprog", None)
    off, on = wcs
    assert off["gate_key_reads"] == off["propagated"]
    assert off["gate_coef_rw"] == off["anticommuting"]
    for k in ("propagated", "merged", "anticommuting", "merge_in", "merge_out"):
        assert on[k] == off[k], k
    # a string that the first rotation creates and the second truncates is
    # never stored, and one that dies and returns keeps its slot
    assert on["appended"] <= off["appended"]
    assert on["gate_key_reads"] < off["gate_key_reads"]
    assert on["gate_coef_rw"] <= off["gate_coef_rw"]
    L.pp_set_gate_fusion(3)


def test_fusion_needs_independent_strings(gpu):
    """All pairs of 4 qubits, lexicographic: XX01 XX02 XX03 form one launch;
    XX12 XX13 commute with XX23 but multiply to it, so XX23 starts a new
    launch: 3 launches per sub-layer (2 if dependence were ignored)."""
    from paper_2512_12094_amd import _lib as L, driver
    prog = W.heisenberg_all_to_all(4, 1, 0.1, eps=1e-6, name="s4")
    L.pp_set_gate_fusion(3)
    prog.meta.pop("_dprog", None)
    info = L.pp_program_info(driver.device_program(prog).h)
    prog.meta.pop("_dprog", None)
    assert info["gates"] == 18 and info["gate_launches"] == 9, info
    res = run_program(gpu, prog, 3)
    same(res, run_program(gpu, prog, 1), "s4")
