"""HIP path vs CPU oracle on the same seeded circuits (calls go through the
C ABI).  Sizes are chosen so that the oracle finishes in seconds while the
sets span many 1024-term tiles and a ragged last tile."""
import math

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
    return dict(torch=torch, stream=stream, handle=int(stream.cuda_stream),
                alloc=_lib.TorchAllocator(0))


def run_both(gpu, prog, group=None, max_sub=None, allocator="torch"):
    from paper_2512_12094_amd import driver
    print(f"[case] {prog.name} group={group or prog.group} n={prog.n} "
          f"sublayers={max_sub or len(prog.sublayers)}", flush=True)
    alloc = gpu["alloc"] if allocator == "torch" else None
    res = driver.propagate(prog, group=group, stream=gpu["handle"], allocator=alloc,
                           max_sublayers=max_sub)
    if max_sub is not None:
        ref = O.run_program(prog, group=group, max_sublayers=max_sub)
    else:
        ref = O.run_program(prog, group=group)
    return res, ref


def check(res, ref, prog, eps=None, what=""):
    eps = prog.meta.get("eps", 0.0) if eps is None else eps
    n, skipped = compare_terms(res.terms, ref.terms, eps, what=what)
    compare_expectation(res.expectation, ref.expectation, ref.terms, what=what)
    if skipped == 0:
        assert (res.propagated, res.merged) == (ref.propagated, ref.merged), what
    return n


def test_config1_translation(gpu):
    prog = W.config1()
    res, ref = run_both(gpu, prog)
    assert check(res, ref, prog, what="c1") == 2048


def test_config1_plain(gpu):
    prog = W.config1()
    res, ref = run_both(gpu, prog, group="none")
    assert check(res, ref, prog, what="c1 plain") == 16384


def test_config1_hipmalloc_allocator(gpu):
    prog = W.config1()
    res, ref = run_both(gpu, prog, allocator=None)
    check(res, ref, prog, what="c1 hipMalloc")


@pytest.mark.parametrize("group", ["Zn", "none"])
def test_config2_prefix(gpu, group):
    """Z_32 XXZ ring with eps = 1e-4, weight <= 8, random Bloch state."""
    prog = W.config2()
    res, ref = run_both(gpu, prog, group=group, max_sub=12)
    check(res, ref, prog, what=f"c2 {group}")


def test_config2_full_program_path(gpu):
    """The benchmarked workload at its full size (all 60 sub-layers), in the
    launch configuration bench.py times (one device program, default gate
    fusion and tuning), against the oracle: sets, coefficients, expectation
    and work counters."""
    from paper_2512_12094_amd import driver
    prog = W.config2()
    print("[case] config 2 full program", flush=True)
    res = driver.propagate_program(prog, stream=gpu["handle"], allocator=gpu["alloc"],
                                   keep_terms=True)
    ref = O.run_program(prog)
    check(res, ref, prog, what="c2 full")


@pytest.mark.parametrize("path", ["program", "layers"])
def test_merge_after_full_trotter_layer(gpu, path):
    """Sec. IV's schedule: the tilted-field Ising ring merged only after each
    full Trotter layer (ZZ, Z, X sub-layers), truncation after every
    sub-layer, on the program path and the per-call path."""
    from paper_2512_12094_amd import driver
    prog = W.tilted_ising_ring(10, 3, 0.25, merge="layer", eps=1e-6)
    print(f"[case] ising merge per layer ({path})", flush=True)
    if path == "program":
        res = driver.propagate_program(prog, stream=gpu["handle"], allocator=gpu["alloc"],
                                       keep_terms=True)
    else:
        res = driver.propagate(prog, stream=gpu["handle"], allocator=gpu["alloc"])
    ref = O.run_program(prog)
    check(res, ref, prog, what=f"ising per layer {path}")


def test_translation_wide_keys(gpu):
    """n = 48 > 32: merge keys do not fit 64 bits (hash + owner compare)."""
    prog = W.xxz_ring(48, 2, 0.3, 1.4, eps=1e-6, obs=W.sum_ring_pairs(48, "X"),
                      bloch=W.random_bloch(48), name="z48")
    res, ref = run_both(gpu, prog)
    check(res, ref, prog, what="z48")


def test_translation_n64_wide(gpu):
    prog = W.xxz_ring(64, 1, 0.2, 0.7, eps=1e-5, wmax=6, name="z64")
    res, ref = run_both(gpu, prog)
    check(res, ref, prog, what="z64")


def test_permutation_config3_prefix(gpu):
    """S_64 all-to-all Heisenberg, noise p = 1e-3, eps = 1e-5: the first two
    sub-layers in Heisenberg order (the second grows to ~6e5 terms)."""
    prog = W.config3()
    res, ref = run_both(gpu, prog, max_sub=2)
    check(res, ref, prog, what="c3")


def test_permutation_two_words(gpu):
    """n = 100: strings span two 64-bit words."""
    prog = W.heisenberg_all_to_all(100, 1, 0.01, eps=1e-4, p=2e-3,
                                   obs=W.sum_single(100, "X", 0.01), bloch=W.random_bloch(5),
                                   name="s100")
    res, ref = run_both(gpu, prog, max_sub=2)
    check(res, ref, prog, what="s100")


def test_plain_two_words(gpu):
    prog = W.xxz_ring(70, 1, 0.3, 1.1, eps=1e-3, obs=W.sum_ring_pairs(70, "Z"),
                      group="none", name="plain70")
    res, ref = run_both(gpu, prog)
    check(res, ref, prog, what="plain70")


@pytest.mark.parametrize("group", ["Zn", "none"])
def test_noise_damping(gpu, group):
    prog = W.xxz_ring(12, 3, 0.4, 0.8, p=0.03, eps=1e-7, obs=W.sum_ring_pairs(12, "Y"),
                      bloch=W.random_bloch(12), name="noisy12")
    res, ref = run_both(gpu, prog, group=group)
    check(res, ref, prog, what=f"noise {group}")


def test_single_qubit_gates_ising(gpu):
    """Tilted-field Ising ring (RZZ bonds, RZ and RX fields)."""
    prog = W.tilted_ising_ring(9, 4, 0.25)
    res, ref = run_both(gpu, prog)
    check(res, ref, prog, what="ising9")
    neck = sum(4 ** math.gcd(j, 9) for j in range(1, 10)) // 9
    assert len(res.terms) <= neck - 1


def test_s2_invariant(gpu):
    n = 10
    prog = W.heisenberg_all_to_all(n, 2, 0.3, obs=W.total_spin_squared(n), bloch=W.PLUS_STATE,
                                   name="s2_10")
    res, ref = run_both(gpu, prog)
    check(res, ref, prog, what="s2")
    assert abs(res.expectation - n * (n + 2) / 4) < 1e-10


def test_edge_observables(gpu):
    from paper_2512_12094_amd import driver
    print("[case] edge observables", flush=True)
    for obs, want in (([], 0.0), ([(0, 0, 2.5)], 2.5), ([(1, 0, 1.0), (1, 0, -1.0)], 0.0)):
        prog = W.xxz_ring(8, 1, 0.3, 1.0, obs=obs, name="edge")
        res = driver.propagate(prog, stream=gpu["handle"], allocator=gpu["alloc"])
        ref = O.run_program(prog)
        compare_terms(res.terms, ref.terms, what="edge")
        assert abs(res.expectation - want) < 1e-12


def test_angles_zero_and_pi(gpu):
    """theta = 0 keeps exact-zero children; theta = pi flips anticommuting terms."""
    for th in (0.0, math.pi):
        prog = W.xxz_ring(6, 1, th, 1.0, obs=W.sum_single(6, "X") + W.sum_ring_pairs(6, "Z"),
                          bloch=W.random_bloch(3), name=f"theta{th}")
        res, ref = run_both(gpu, prog, group="none")
        check(res, ref, prog, what=f"theta={th}")


def test_repeat_runs_agree(gpu):
    from paper_2512_12094_amd import driver
    print("[case] repeat", flush=True)
    prog = W.config2()
    a = driver.propagate(prog, stream=gpu["handle"], allocator=gpu["alloc"], max_sublayers=9)
    b = driver.propagate(prog, stream=gpu["handle"], allocator=gpu["alloc"], max_sublayers=9)
    compare_terms(a.terms, b.terms, prog.meta["eps"], rel=1e-14, what="repeat")


def test_errors(gpu):
    from paper_2512_12094_amd import _lib as L
    from paper_2512_12094_amd import driver
    print("[case] errors", flush=True)
    prog = W.config1()
    ps = driver.PauliSet.from_program(prog, stream=gpu["handle"], allocator=gpu["alloc"])
    before = ps.as_dict()
    # not closed under translations: one bond only
    with pytest.raises(L.PPError) as e:
        L.pp_apply_layer(ps.h, [3], [0], [0.1], 1)
    assert e.value.code == -2
    with pytest.raises(L.PPError) as e:
        L.pp_apply_layer(ps.h, [1 << 9], [0], [0.1], 1)      # bit >= n
    assert e.value.code == -1
    with pytest.raises(L.PPError) as e:
        L.pp_apply_layer(ps.h, [3], [0], [0.1], 1, merge_every=2)
    assert e.value.code == -1
    assert ps.as_dict() == before                             # unchanged
    ps.close()


def test_capacity_limit(gpu):
    from paper_2512_12094_amd import _lib as L
    from paper_2512_12094_amd import driver
    print("[case] capacity", flush=True)
    prog = W.config1().with_group("none")
    ps = driver.PauliSet.from_program(prog, stream=gpu["handle"], allocator=gpu["alloc"])
    L.pp_set_max_terms(ps.h, 5000)
    layers = driver.heisenberg_layers(prog)
    before = after = None
    with pytest.raises(L.PPError) as e:
        for la in layers:
            before = (ps.as_dict(), L.pp_work_counters(ps.h))
            ps.apply_layer(la)
    assert e.value.code == -4
    assert "as before the call" in str(e.value)
    # the failed call left the handle exactly as it was before it
    after = (ps.as_dict(), L.pp_work_counters(ps.h))
    assert after[1] == before[1]
    assert after[0] == before[0]
    # and the handle keeps working: the same layer under a larger limit
    L.pp_set_max_terms(ps.h, 0)
    ps.apply_layer(la)
    assert ps.num_terms() > 0
    ps.close()


def test_batch_matches_solo(gpu):
    """Batched form: every instance equals its own oracle run."""
    from paper_2512_12094_amd import driver
    print("[case] batch", flush=True)
    rng = np.random.default_rng(11)
    progs = []
    for k in range(6):
        n = int(rng.choice([8, 12, 16, 24, 40]))
        progs.append(W.xxz_ring(n, int(rng.integers(1, 4)), float(rng.uniform(0.05, 0.3)),
                                float(rng.uniform(0.5, 2)), eps=1e-6, name=f"b{k}_n{n}"))
    progs.append(W.heisenberg_all_to_all(20, 1, 0.1, eps=1e-5, p=1e-3, name="b_s20"))
    progs.append(W.xxz_ring(10, 2, 0.2, 1.0, eps=0.0, group="none", name="b_plain10"))
    e, sets, dprogs, wall = driver.batch_propagate(progs, gpu["handle"], gpu["alloc"])
    for p, ei, s in zip(progs, e, sets):
        ref = O.run_program(p)
        compare_terms(s.as_dict(), ref.terms, p.meta.get("eps", 0.0), what=p.name)
        compare_expectation(ei, ref.expectation, ref.terms, what=p.name)
        assert s.counters() == (ref.propagated, ref.merged), p.name
    for s in sets:
        s.close()
    for d in dprogs:
        d.close()


def heisenberg_prefix(prog, k):
    """The first k sub-layers in Heisenberg order = the last k in time."""
    return W.Program(prog.name + f"[:{k}]", prog.n, prog.group, prog.obs,
                     prog.sublayers[len(prog.sublayers) - k:], prog.bloch, dict(prog.meta))


@pytest.mark.parametrize("which", ["c2", "c2plain", "c3", "z48"])
def test_program_path_matches_oracle(gpu, which):
    """One device program per propagation (pp_batch_run with one instance):
    all sub-layers queued ahead, growth handled mid-program."""
    from paper_2512_12094_amd import driver
    if which == "c2":
        prog, group = heisenberg_prefix(W.config2(), 12), None
    elif which == "c2plain":
        prog, group = heisenberg_prefix(W.config2(), 9), "none"
    elif which == "c3":
        prog, group = heisenberg_prefix(W.config3(), 2), None
    else:
        prog, group = W.xxz_ring(48, 2, 0.3, 1.4, eps=1e-6, obs=W.sum_ring_pairs(48, "X"),
                                 bloch=W.random_bloch(48), name="z48"), None
    print(f"[case] program {prog.name} group={group or prog.group}", flush=True)
    res = driver.propagate_program(prog, group=group, stream=gpu["handle"],
                                   allocator=gpu["alloc"], keep_terms=True)
    ref = O.run_program(prog, group=group)
    check(res, ref, prog, what=f"program {which}")


# ----------------------------------------------------------------------------
# Dihedral group D_n
# ----------------------------------------------------------------------------
def test_dihedral_config1(gpu):
    """Config 1's circuit merged under D_8: untruncated, so the set is fixed
    by integer algebra and must match bit for bit."""
    prog = W.config1().with_group("Dn")
    res, ref = run_both(gpu, prog)
    n = check(res, ref, prog, what="c1 Dn")
    assert n == len(ref.terms) and set(res.terms) == set(ref.terms)


def test_dihedral_config2_prefix(gpu):
    prog = W.config2().with_group("Dn")
    res, ref = run_both(gpu, prog, max_sub=12)
    check(res, ref, prog, what="c2 Dn")


def test_dihedral_wide_and_program_path(gpu):
    """n = 48 (keys wider than 64 bits) through the one-program path."""
    from paper_2512_12094_amd import driver
    prog = W.xxz_ring(48, 2, 0.3, 1.4, eps=1e-6, obs=W.sum_ring_pairs(48, "X"),
                      bloch=W.random_bloch(48), group="Dn", name="d48")
    print("[case] program d48 Dn", flush=True)
    res = driver.propagate_program(prog, stream=gpu["handle"], allocator=gpu["alloc"],
                                   keep_terms=True)
    ref = O.run_program(prog)
    check(res, ref, prog, what="d48")


def test_dihedral_rejects_chiral_layer(gpu):
    """X_b Y_{b+1} on every bond is closed under translations but its
    reflection Y_b X_{b+1} is absent: PP_ENOTSYM under D_n, fine under Z_n."""
    from paper_2512_12094_amd import _lib as L
    n = 8
    gx = np.array([[(1 << b) | (1 << ((b + 1) % n))] for b in range(n)], dtype=np.uint64)
    gz = np.array([[1 << ((b + 1) % n)] for b in range(n)], dtype=np.uint64)
    th = np.full(n, 0.1)
    x, z = W.one_site("Z", 0)
    for group, ok in (("Zn", True), ("Dn", False)):
        h = L.pp_create(n, group, np.array([[x]], dtype=np.uint64),
                        np.array([[z]], dtype=np.uint64), np.array([1.0]), gpu["handle"],
                        gpu["alloc"])
        try:
            L.pp_apply_layer(h, gx, gz, th, 1)
            assert ok, group
        except L.PPError as e:
            assert not ok and e.code == -2, (group, e)
        finally:
            L.pp_destroy(h)


def test_tilted_ising_saturates_below_necklace_count(gpu):
    """Tilted-field Ising ring (Sec. IV), untruncated, merged after every
    sub-layer: the GPU's set after every layer matches the oracle's size and
    stays below the necklace count minus one (the identity is never produced
    from a traceless observable), and the final set matches exactly."""
    from paper_2512_12094_amd import driver
    n = 8
    prog = W.tilted_ising_ring(n, 8, 0.4)
    print("[case] tilted Ising n=8", flush=True)
    res = driver.propagate(prog, stream=gpu["handle"], allocator=gpu["alloc"],
                           record_sizes=True)
    ref = O.run_program(prog)
    neck = sum(4 ** math.gcd(j, n) for j in range(1, n + 1)) // n
    assert max(res.sizes) <= neck - 1 and (0, 0) not in res.terms
    assert res.sizes == ref.sizes and res.sizes[-1] == len(ref.terms)
    n_cmp = check(res, ref, prog, what="ising")
    assert n_cmp == len(ref.terms)


# ----------------------------------------------------------------------------
# 2D translations of a torus
# ----------------------------------------------------------------------------
def test_torus_untruncated_3x3(gpu):
    prog = W.power_law_xxz_torus(3, 3, 1, 0.2, bloch=W.random_bloch(9))
    res, ref = run_both(gpu, prog)
    n = check(res, ref, prog, what="torus 3x3")
    assert n == len(ref.terms) and set(res.terms) == set(ref.terms)


def test_torus_truncated_4x4(gpu):
    prog = W.power_law_xxz_torus(4, 4, 1, 0.1, eps=1e-4, bloch=W.random_bloch(16))
    res, ref = run_both(gpu, prog)
    check(res, ref, prog, what="torus 4x4")


def test_torus_6x6_wide_program_path(gpu):
    """n = 36: keys wider than 64 bits; one device program."""
    from paper_2512_12094_amd import driver
    prog = W.power_law_xxz_torus(6, 6, 1, 0.05, eps=1e-3, bloch=W.random_bloch(36))
    print("[case] program torus 6x6", flush=True)
    res = driver.propagate_program(prog, stream=gpu["handle"], allocator=gpu["alloc"],
                                   keep_terms=True)
    ref = O.run_program(prog)
    check(res, ref, prog, what="torus 6x6")


def test_torus_rejects_row_only_layer(gpu):
    """XX on the bonds of row 0 only: closed under x shifts, not under y."""
    from paper_2512_12094_amd import _lib as L
    lx, ly = 4, 3
    gx = np.array([[(1 << a) | (1 << ((a + 1) % lx))] for a in range(lx)], dtype=np.uint64)
    gz = np.zeros((lx, 1), dtype=np.uint64)
    x, z = W.one_site("Z", 0)
    h = L.pp_create_torus(lx, ly, np.array([[x]], dtype=np.uint64),
                          np.array([[z]], dtype=np.uint64), np.array([1.0]), gpu["handle"],
                          gpu["alloc"])
    try:
        with pytest.raises(L.PPError) as e:
            L.pp_apply_layer(h, gx, gz, np.full(lx, 0.1), 1)
        assert e.value.code == -2
    finally:
        L.pp_destroy(h)


# ----------------------------------------------------------------------------
# Any permutation group given by its element list
# ----------------------------------------------------------------------------
def test_explicit_dihedral_list_equals_dihedral_handle(gpu):
    from paper_2512_12094_amd import driver
    base = W.config1()
    prog = W.with_explicit_group(base, W.elements_dihedral(8))
    print("[case] explicit D_8 list", flush=True)
    g = driver.propagate(prog, stream=gpu["handle"], allocator=gpu["alloc"])
    d = driver.propagate(base, group="Dn", stream=gpu["handle"], allocator=gpu["alloc"])
    assert g.terms == d.terms and g.expectation == d.expectation
    ref = O.run_program(prog)
    check(g, ref, prog, what="explicit D8")


def test_explicit_symmetric_group_equals_permutation_handle(gpu):
    """S_5 as its 120 elements: the same representatives as Algorithm 3."""
    from paper_2512_12094_amd import driver
    base = W.heisenberg_all_to_all(5, 2, 0.2, obs=W.sum_single(5, "Z"), bloch=W.random_bloch(5))
    prog = W.with_explicit_group(base, W.elements_symmetric(5))
    print("[case] explicit S_5 list", flush=True)
    g = driver.propagate(prog, stream=gpu["handle"], allocator=gpu["alloc"])
    p = driver.propagate(base, stream=gpu["handle"], allocator=gpu["alloc"])
    assert g.terms == p.terms and g.expectation == p.expectation


def test_explicit_cyclic_group_on_a_symmetrised_circuit(gpu):
    """A cyclic group of order 6 on 5 qubits, (0 1 2)(3 4): a circuit made
    closed under it by taking every gate's images; vs the oracle."""
    from paper_2512_12094_amd import driver
    gen = [1, 2, 0, 4, 3]
    perms, cur = [], list(range(5))
    for _ in range(6):
        perms.append(cur)
        cur = [cur[gen[q]] for q in range(5)]
    seeds = [W.Gate(*W.two_site("X", 0, 3), 0.3), W.Gate(*W.two_site("Z", 1, 4), 0.2),
             W.Gate(*W.one_site("Y", 0), 0.25)]
    subs = [W.SubLayer(W.symmetrize([s], perms)) for s in seeds] * 2
    obs = [(*W.one_site("Z", q), 1.0) for q in range(5)]
    prog = W.Program("c6", 5, "G", obs, subs, W.random_bloch(7), dict(perms=perms))
    print("[case] explicit cyclic group of order 6", flush=True)
    res = driver.propagate(prog, stream=gpu["handle"], allocator=gpu["alloc"])
    ref = O.run_program(prog)
    n = check(res, ref, prog, what="c6")
    assert n == len(ref.terms)
    plain = O.run_program(prog, group="none", keep_terms=False)
    assert abs(res.expectation - plain.expectation) < 1e-12 * max(1, abs(plain.expectation))


def test_explicit_group_rejects_open_layer(gpu):
    from paper_2512_12094_amd import _lib as L
    perms = W.elements_dihedral(6)
    x, z = W.one_site("Z", 0)
    h = L.pp_create_group(6, perms, np.array([[x]], dtype=np.uint64),
                          np.array([[z]], dtype=np.uint64), np.array([1.0]), gpu["handle"],
                          gpu["alloc"])
    gx = np.array([[W.two_site("X", 0, 1)[0]]], dtype=np.uint64)
    try:
        with pytest.raises(L.PPError) as e:
            L.pp_apply_layer(h, gx, np.zeros((1, 1), dtype=np.uint64), np.array([0.1]), 1)
        assert e.value.code == -2
    finally:
        L.pp_destroy(h)
