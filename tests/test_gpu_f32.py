"""FP32 coefficient mode (PP_F32_COMPENSATED) against the FP64 oracle, by
the FP32 rules of tests/parity.py: the one-instance program path, the
per-call path, growth of the store, and the batched form (each instance
equal to its FP32 solo run, bitwise)."""
import pytest

from oracle import oracle as O
from paper_2512_12094_amd import workloads as W
from tests.parity import REL32, compare_expectation, compare_terms_f32, f32_error_report

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
    return dict(torch=torch, stream=stream, handle=int(stream.cuda_stream),
                alloc=_lib.TorchAllocator(0))


def prefix(prog, k):
    return W.Program(prog.name + f"[:{k}]", prog.n, prog.group, prog.obs,
                     prog.sublayers[len(prog.sublayers) - k:], prog.bloch, dict(prog.meta))


def check(res, ref, prog, what):
    n, skipped = compare_terms_f32(res.terms, ref.terms, prog.meta.get("eps", 0.0), what=what)
    rep = f32_error_report(res.terms, ref.terms)
    print(f"[f32] {what}: relative error by decade {rep['rel_by_decade']}, worst "
          f"{rep['worst_roundings']:.2f} roundings of max|c|, {skipped} near eps skipped",
          flush=True)
    compare_expectation(res.expectation, ref.expectation, ref.terms, rel=REL32, what=what)
    assert (res.propagated, res.merged) == (ref.propagated, ref.merged), what
    return n


CASES = {
    "c1": lambda: W.config1(),                          # no truncation: sets bit-exact
    "c2": lambda: prefix(W.config2(), 30),
    "c3": lambda: prefix(W.config3(), 2),               # grows to ~6e5 strings
    "z48": lambda: W.xxz_ring(48, 2, 0.3, 1.4, eps=1e-6, obs=W.sum_ring_pairs(48, "X"),
                              bloch=W.random_bloch(48), name="z48"),
}


@pytest.mark.parametrize("which", list(CASES))
def test_f32_program_path(gpu, which):
    from paper_2512_12094_amd import driver
    prog = CASES[which]()
    print(f"[case] f32 program {prog.name}", flush=True)
    res = driver.propagate_program(prog, stream=gpu["handle"], allocator=gpu["alloc"],
                                   keep_terms=True, dtype="f32")
    ref = O.run_program(prog)
    n = check(res, ref, prog, f"f32 {which}")
    if which == "c1":
        assert set(res.terms) == set(ref.terms) and n == len(ref.terms)


def test_f32_per_call_path(gpu):
    """pp_apply_layer / pp_merge_canonicalize / pp_truncate / pp_expectation
    on an FP32 handle."""
    from paper_2512_12094_amd import driver
    prog = prefix(W.config2(), 9)
    print("[case] f32 per-call c2[:9]", flush=True)
    res = driver.propagate(prog, stream=gpu["handle"], allocator=gpu["alloc"], dtype="f32")
    ref = O.run_program(prog)
    check(res, ref, prog, "f32 calls")


def test_f32_batch_equals_solo(gpu):
    from paper_2512_12094_amd import driver
    progs = [prefix(p, 6) for p in W.config4()[:8]]
    print("[case] f32 batch of", [p.n for p in progs], flush=True)
    e, sets, dprogs, _ = driver.batch_propagate(progs, gpu["handle"], gpu["alloc"], dtype="f32")
    for p, ei, s in zip(progs, e, sets):
        ref = O.run_program(p)
        compare_terms_f32(s.as_dict(), ref.terms, p.meta["eps"], what=p.name)
        compare_expectation(float(ei), ref.expectation, ref.terms, rel=REL32, what=p.name)
        solo = driver.propagate_program(p, stream=gpu["handle"], allocator=gpu["alloc"],
                                        dtype="f32")
        assert float(ei) == solo.expectation, (p.name, ei, solo.expectation)
        s.close()
    for d in dprogs:
        d.close()
