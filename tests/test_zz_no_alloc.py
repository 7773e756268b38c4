"""pp_expectation_noalloc (the allocation-free variant of pp_expectation)
against pp_expectation itself, through the C ABI, on two calls in a row: a
Z_32 ring propagated through several sub-layers and stopped right after a
sub-layer's truncating gates (so the store holds dead entries), then a smaller Z_8 ring.
Both entry points form the same products and sum them exactly, so the
values must agree bitwise; the variant must not call the handle's
allocator.  Algorithm 1 step 3."""
import numpy as np
import pytest

from paper_2512_12094_amd import workloads as W

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
    calls = {"alloc": 0}
    alloc = _lib.TorchAllocator(0)
    inner = alloc._alloc

    def counting(nbytes, stream_, ctx):
        calls["alloc"] += 1
        return inner(nbytes, stream_, ctx)

    alloc._alloc_counting = _lib.ALLOC_FN(counting)
    alloc.struct = _lib.PPAllocator(alloc._alloc_counting, alloc._free, None)
    return dict(torch=torch, stream=stream, handle=int(stream.cuda_stream), alloc=alloc,
                calls=calls)


def both(gpu, h, bloch):
    from paper_2512_12094_amd import _lib as L
    want = L.pp_expectation(h, bloch)
    before = gpu["calls"]["alloc"]
    got = L.pp_expectation_noalloc(h, bloch)
    assert gpu["calls"]["alloc"] == before, "the allocation-free call used the allocator"
    again = L.pp_expectation_noalloc(h, bloch)
    return want, got, again


def test_noalloc_expectation_matches_pp_expectation(gpu):
    from paper_2512_12094_amd import _lib as L
    from paper_2512_12094_amd import driver
    # call 1: Z_32 XXZ ring, 8 sub-layers, then a 9th sub-layer's gates with
    # their truncation but no merge (the store keeps the truncated entries)
    prog = W.config2()
    layers = driver.heisenberg_layers(prog)
    ps = driver.PauliSet.from_program(prog, None, gpu["handle"], gpu["alloc"])
    driver.run_layers(ps, layers[:8])
    ps.apply_layer(layers[8])
    n1 = L.pp_num_terms(ps.h)
    print(f"[case] noalloc expectation, Z_32 ring, {n1} live terms", flush=True)
    for bloch in (prog.bloch, (0.0, 0.0, 1.0), (0.6, -0.48, 0.64)):
        want, got, again = both(gpu, ps.h, bloch)
        assert got == want and again == want, (bloch, got, want, again)
    ps.close()
    # call 2: a smaller input (Z_8 ring of config 1)
    prog8 = W.config1()
    ps8 = driver.PauliSet.from_program(prog8, None, gpu["handle"], gpu["alloc"])
    driver.run_layers(ps8, driver.heisenberg_layers(prog8)[:2])
    n2 = L.pp_num_terms(ps8.h)
    assert 0 < n2 < n1
    print(f"[case] noalloc expectation, Z_8 ring, {n2} live terms", flush=True)
    for bloch in (prog8.bloch, (0.3, 0.4, np.sqrt(1 - 0.25))):
        want, got, again = both(gpu, ps8.h, bloch)
        assert got == want and again == want, (bloch, got, want, again)
    ps8.close()


def test_noalloc_expectation_fp32_store(gpu):
    """FP32 coefficients: the same widened products on both entry points."""
    from paper_2512_12094_amd import driver
    prog = W.config1()
    ps = driver.PauliSet.from_program(prog, None, gpu["handle"], gpu["alloc"], dtype="f32")
    driver.run_layers(ps, driver.heisenberg_layers(prog)[:4])
    print("[case] noalloc expectation, FP32 store", flush=True)
    want, got, again = both(gpu, ps.h, (0.1, 0.2, 0.97))
    assert got == want and again == want
    ps.close()
