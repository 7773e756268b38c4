"""Pins for the CPU oracle: facts fixed by the paper or by the mathematics,
checked without using the oracle's own formulas.

* Pauli products vs 2x2 / 2^n matrix products (symplectic form, App. E.2).
* Orbit counts vs the Burnside / necklace / stars-and-bars closed forms and
  the paper's printed Z_3 example (App. B).
* Canonical forms vs brute force over the whole orbit with an independent
  integer encoding (Definition "lowest integer representation", App. E.2;
  Algorithms 2 and 3).
* Propagation vs dense 2^n Heisenberg evolution U^dag O U (Prop. 1 rule,
  Algorithm 1, Theorem 1), plain and merged.
* Noise vs a density-matrix simulation.
"""
import itertools
import math
import os
import random

import numpy as np
import pytest

from oracle import oracle as O
from paper_2512_12094_amd import workloads as W
from tests import dense

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden_lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [l.split() for l in f if l.strip() and not l.startswith("#")]


# ----------------------------------------------------------------------------
# independent helpers (plain Python, no oracle code)
# ----------------------------------------------------------------------------
DIGIT = {"I": 0, "X": 1, "Y": 2, "Z": 3}   # App. E.2: I->00 X->01 Y->10 Z->11


def int_value(x, z, n):
    """sum_q digit(q) 4^q (qubit q is the base-4 digit of weight 4^q)."""
    s = W.to_letters(x, z, n)
    return sum(DIGIT[ch] * 4 ** q for q, ch in enumerate(s))


def join(words):
    """Row of uint64 words (word w holds qubits 64w..64w+63) -> one integer."""
    return sum(int(v) << (64 * w) for w, v in enumerate(words))


def rotate_letters(s, j):
    """T^j: qubit q takes the letter of qubit q+j (T.(IXI) = XII)."""
    n = len(s)
    return "".join(s[(q + j) % n] for q in range(n))


def random_string(rng, n, weight=None):
    letters = ["I"] * n
    qs = range(n) if weight is None else rng.sample(range(n), weight)
    for q in qs:
        letters[q] = rng.choice("IXYZ" if weight is None else "XYZ")
    return "".join(letters)


# ----------------------------------------------------------------------------
# Pauli algebra
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 3])
def test_products_match_matrices(n):
    strings = ["".join(t) for t in itertools.product("IXYZ", repeat=n)]
    mats = {s: dense.pauli_matrix(*W.from_letters(s), n) for s in strings}
    for a in strings:
        for b in strings:
            k, rx, rz = O.multiply(n, W.from_letters(a), W.from_letters(b))
            expect = mats[a] @ mats[b]
            got = (1j ** k) * dense.pauli_matrix(rx, rz, n)
            assert np.allclose(expect, got), (a, b, k)


def test_products_wide_strings():
    """Letter-wise phases also hold across the 64-qubit word boundary."""
    rng = random.Random(3)
    n = 100
    for _ in range(50):
        a, b = random_string(rng, n), random_string(rng, n)
        k, rx, rz = O.multiply(n, W.from_letters(a), W.from_letters(b))
        # per-letter products from the 2x2 matrices
        kk, out = 0, []
        for la, lb in zip(a, b):
            m = dense.SIGMA[la] @ dense.SIGMA[lb]
            for lc in "IXYZ":
                for ph in range(4):
                    if np.allclose(m, (1j ** ph) * dense.SIGMA[lc]):
                        out.append(lc)
                        kk += ph
        assert W.to_letters(rx, rz, n) == "".join(out)
        assert k == kk % 4


def test_dense_phase_permutation_matches_kron():
    for n in (1, 2, 3):
        N = 2 ** n
        k = np.arange(N)
        for x in range(N):
            for z in range(N):
                P = dense.pauli_matrix(x, z, n)
                ph = dense.pauli_phase_perm(x, z, n)
                assert np.allclose(P[k ^ x, k], ph)
                Q = P.copy()
                Q[k ^ x, k] = 0
                assert np.allclose(Q, 0)


# ----------------------------------------------------------------------------
# Orbit counts (Burnside) and the paper's worked examples
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("group,n,count", [(g, int(n), int(c)) for g, n, c in
                                           golden_lines("representative_counts.txt")])
def test_representative_counts(group, n, count):
    reps = set()
    for s in itertools.product("IXYZ", repeat=n):
        reps.add(O.canon(n, group, *W.from_letters("".join(s))))
    assert len(reps) == count
    # and the closed forms of App. B agree with the fixture
    if group == "Zn":
        assert sum(4 ** math.gcd(j, n) for j in range(1, n + 1)) // n == count
    else:
        assert math.comb(n + 3, 3) == count


def test_necklace_count_n8_and_prime_formula():
    n = 8
    reps = set()
    for s in itertools.product("IXYZ", repeat=n):
        reps.add(O.canon(n, "Zn", *W.from_letters("".join(s))))
    assert len(reps) == 8230
    for p in (3, 5, 7, 11, 13):   # prime n: (4^n + 4(n-1)) / n
        assert sum(4 ** math.gcd(j, p) for j in range(1, p + 1)) == 4 ** p + 4 * (p - 1)


def test_z3_example_list_is_a_complete_set():
    """The 24 strings the paper lists for Z_3 are pairwise inequivalent, so
    they form a complete set of representatives (the paper's list is not the
    lowest-integer set; only its size and completeness are pinned)."""
    strings = [s for line in golden_lines("z3_representatives.txt") for s in line]
    assert len(strings) == 24
    reps = {O.canon(3, "Zn", *W.from_letters(s)) for s in strings}
    assert len(reps) == 24


def test_group_action_examples():
    for row in golden_lines("orbit_examples.txt"):
        if row[0] == "translate":
            assert rotate_letters(row[1], 1) == row[2]
            # the oracle's representative is invariant under that move
            assert O.canon(3, "Zn", *W.from_letters(row[1])) == \
                O.canon(3, "Zn", *W.from_letters(row[2]))
        elif row[0] == "orbit":
            s = row[1]
            orbit = {rotate_letters(s, j) for j in range(len(s))}
            assert orbit == set(row[2].split(","))
            reps = {O.canon(len(s), "Zn", *W.from_letters(t)) for t in orbit}
            assert len(reps) == 1
        elif row[0] == "weight":
            # weight truncation: a string of weight w survives wmax = w only
            n = len(row[1])
            for wmax, survives in ((int(row[2]), True), (int(row[2]) - 1, False)):
                o = O.Oracle(n, "none")
                o.add(*W.from_letters(row[1]), 1.0)
                o.truncate(0.0, wmax)
                assert (o.size() == 1) == survives


# ----------------------------------------------------------------------------
# Canonical forms vs brute force (independent integer encoding)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("n", [5, 8, 17, 31, 32, 33, 64, 65, 100])
def test_translation_representative_is_orbit_minimum(n):
    rng = random.Random(n)
    for trial in range(40):
        s = random_string(rng, n, None if trial % 2 else rng.randint(0, min(n, 9)))
        rx, rz = O.canon(n, "Zn", *W.from_letters(s))
        orbit = [rotate_letters(s, j) for j in range(n)]
        best = min(orbit, key=lambda t: int_value(*W.from_letters(t), n))
        assert W.to_letters(rx, rz, n) == best
        # idempotent (Observation 1) and invariant under every translation
        assert O.canon(n, "Zn", rx, rz) == (rx, rz)
        j = rng.randrange(n)
        assert O.canon(n, "Zn", *W.from_letters(orbit[j])) == (rx, rz)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_permutation_representative_is_orbit_minimum(n):
    for s in itertools.product("IXYZ", repeat=n):
        s = "".join(s)
        rx, rz = O.canon(n, "Sn", *W.from_letters(s))
        best = min({"".join(p) for p in itertools.permutations(s)},
                   key=lambda t: int_value(*W.from_letters(t), n))
        assert W.to_letters(rx, rz, n) == best


def test_permutation_representative_wide():
    rng = random.Random(11)
    for n in (64, 96, 128):
        for _ in range(20):
            s = random_string(rng, n)
            rx, rz = O.canon(n, "Sn", *W.from_letters(s))
            r = W.to_letters(rx, rz, n)
            # Z^{nZ} Y^{nY} X^{nX} I^{rest}, qubit 0 first
            nz, ny, nx = s.count("Z"), s.count("Y"), s.count("X")
            assert r == "Z" * nz + "Y" * ny + "X" * nx + "I" * (n - nx - ny - nz)
            perm = list(s)
            rng.shuffle(perm)
            assert O.canon(n, "Sn", *W.from_letters("".join(perm))) == (rx, rz)


def test_int_order_matches_integer_encoding():
    rng = random.Random(5)
    for n in (3, 40, 70):
        for _ in range(200):
            a, b = random_string(rng, n), random_string(rng, n)
            A, B = W.from_letters(a), W.from_letters(b)
            assert O.int_less(n, A, B) == (int_value(*A, n) < int_value(*B, n))


@pytest.mark.parametrize("n,group", [(8, "Zn"), (40, "none"), (70, "none"), (12, "Sn")])
def test_export_is_key_sorted(n, group):
    """The exported set is one record per representative, in ascending order
    of the App. E.2 integer (computed here from the letters)."""
    rng = random.Random(n)
    o = O.Oracle(n, group)
    for _ in range(300):
        o.add(*W.from_letters(random_string(rng, n)), rng.uniform(-1, 1))
    o.merge()
    x, z, c = o.export()
    keys = [int_value(join(x[i]), join(z[i]), n) for i in range(len(c))]
    assert len(keys) > 100
    assert all(a < b for a, b in zip(keys, keys[1:]))


# ----------------------------------------------------------------------------
# Propagation vs dense evolution
# ----------------------------------------------------------------------------
def small_ring(n, steps=2, theta=0.3, delta=1.7, obs=None, bloch=W.ZERO_STATE, p=0.0):
    return W.xxz_ring(n, steps, theta, delta, obs=obs, bloch=bloch, p=p)


def orbit_sums(coeffs, n, group):
    sums = {}
    for (x, z), c in coeffs.items():
        r = O.canon(n, group, x, z)
        sums[r] = sums.get(r, 0.0) + c
    return sums


def assert_terms_match(got: dict, want: dict, tol=1e-12):
    scale = max([abs(v) for v in want.values()] + [1.0])
    keys = set(got) | set(want)
    for k in keys:
        a, b = got.get(k, 0.0), want.get(k, 0.0)
        assert abs(a - b) <= tol * scale, (k, a, b)


@pytest.mark.parametrize("n", [3, 4, 5])
def test_plain_pp_matches_dense(n):
    prog = small_ring(n, obs=[(*W.one_site("Z", 0), 1.0), (*W.two_site("X", 0, 1), 0.5)])
    res = O.run_program(prog, group="none")
    Od = dense.heisenberg(prog)
    coeffs = dense.pauli_coefficients(Od, n)
    want = {k: v.real for k, v in coeffs.items() if abs(v) > 1e-14}
    assert max(abs(v.imag) for v in coeffs.values()) < 1e-12
    assert_terms_match(res.terms, want)
    assert abs(res.expectation - dense.expectation(Od, prog.bloch, n)) < 1e-12


@pytest.mark.parametrize("n,group,prog_fn", [
    (4, "Zn", lambda n: small_ring(n, obs=W.sum_single(n, "Z"))),
    (5, "Zn", lambda n: small_ring(n, obs=W.sum_ring_pairs(n, "X"), bloch=W.random_bloch(9))),
    (4, "Sn", lambda n: W.heisenberg_all_to_all(n, 2, 0.2, obs=W.sum_single(n, "Z"))),
    (5, "Sn", lambda n: W.heisenberg_all_to_all(n, 1, 0.3, obs=W.total_spin_squared(n),
                                                 bloch=W.PLUS_STATE)),
])
def test_symmetry_pp_matches_dense_orbit_sums(n, group, prog_fn):
    prog = prog_fn(n)
    res = O.run_program(prog, group=group)
    Od = dense.heisenberg(prog)
    coeffs = {k: v.real for k, v in dense.pauli_coefficients(Od, n).items()}
    want = {k: v for k, v in orbit_sums(coeffs, n, group).items()}
    # every representative the oracle keeps has the dense orbit sum; those it
    # never produced have orbit sum zero
    assert_terms_match(res.terms, {k: v for k, v in want.items() if abs(v) > 1e-13})
    assert abs(res.expectation - dense.expectation(Od, prog.bloch, n)) < 1e-12


def test_config1_against_dense_256():
    """Config 1 exactly: Z_8 ring, 6 steps of RXX/RYY/RZZ(0.1), O = sum Z_i,
    no truncation, merged after every sub-layer, vs 256x256 evolution."""
    prog = W.config1()
    res = O.run_program(prog)
    Od = dense.heisenberg(prog)
    coeffs = {k: v.real for k, v in dense.pauli_coefficients(Od, 8).items()}
    want = orbit_sums(coeffs, 8, "Zn")
    assert_terms_match(res.terms, {k: v for k, v in want.items() if abs(v) > 1e-13})
    e = dense.expectation(Od, prog.bloch, 8)
    assert abs(res.expectation - e) < 1e-12
    plain = O.run_program(prog, group="none")
    assert abs(plain.expectation - e) < 1e-12


def test_theorem1_merged_equals_plain():
    """Theorem 1: with exactly symmetric layers and state, the merged
    propagation gives the plain propagation's expectation (truncation off)."""
    for n, steps in ((9, 3), (10, 2)):
        prog = W.xxz_ring(n, steps, 0.21, 1.3, obs=W.sum_ring_pairs(n, "X"),
                          bloch=W.random_bloch(n))
        a = O.run_program(prog, group="Zn", keep_terms=False)
        b = O.run_program(prog, group="none", keep_terms=False)
        assert abs(a.expectation - b.expectation) < 1e-12 * max(1, abs(b.expectation))
        # Observation 2 / Theorem 2: ceil(N/|G|) <= N_tilde <= N
        assert math.ceil(b.sizes[-1] / n) <= a.sizes[-1] <= b.sizes[-1]
    prog = W.heisenberg_all_to_all(7, 2, 0.15, obs=W.sum_single(7, "Z"),
                                   bloch=W.random_bloch(3))
    a = O.run_program(prog, group="Sn", keep_terms=False)
    b = O.run_program(prog, group="none", keep_terms=False)
    assert abs(a.expectation - b.expectation) < 1e-12 * max(1, abs(b.expectation))
    assert a.sizes[-1] <= b.sizes[-1]


def test_single_gate_closed_forms():
    rng = random.Random(1)
    n = 6
    P = W.from_letters("XYIZIX")
    terms = {}
    for _ in range(30):
        s = random_string(rng, n)
        terms[W.from_letters(s)] = rng.uniform(-1, 1)

    def run(theta):
        o = O.Oracle(n, "none")
        for (x, z), c in terms.items():
            o.add(x, z, c)
        o.apply_gate(*P, theta, 0.0, -1)
        return o.as_dict()

    # identity map; anticommuting terms leave exact-zero children (nothing is
    # dropped with truncation off)
    out = run(0.0)
    assert {k: v for k, v in out.items() if v != 0.0} == terms
    assert all(v == 0.0 for k, v in out.items() if k not in terms)
    # theta = pi: anticommuting Q -> -Q, commuting Q -> Q
    Pm = dense.pauli_matrix(*P, n)
    out = run(math.pi)
    for (x, z), c in terms.items():
        Q = dense.pauli_matrix(x, z, n)
        anti = np.allclose(Pm @ Q, -Q @ Pm)
        assert abs(out[(x, z)] - (-c if anti else c)) < 1e-12
    # theta = pi/2: Clifford, Q -> iPQ for anticommuting Q, sizes preserved
    out = {k: v for k, v in run(math.pi / 2).items() if abs(v) > 1e-12}
    assert len(out) == len(terms)
    for (x, z), c in terms.items():
        Q = dense.pauli_matrix(x, z, n)
        if np.allclose(Pm @ Q, -Q @ Pm):
            M = 1j * Pm @ Q
            hits = [(k, v) for k, v in out.items()
                    if np.allclose(M, dense.pauli_matrix(*k, n)) or
                    np.allclose(M, -dense.pauli_matrix(*k, n))]
            assert len(hits) == 1


def test_saturation_below_necklace_count():
    """Fig. 2 / Example Z_n: untruncated merged counts never exceed the
    number of representatives; a traceless observable never produces the
    identity, so at most necklace - 1 terms."""
    n = 5
    prog = W.tilted_ising_ring(n, 8, 0.4)
    res = O.run_program(prog, keep_terms=True)
    neck = sum(4 ** math.gcd(j, n) for j in range(1, n + 1)) // n
    assert max(res.sizes) <= neck - 1
    assert (0, 0) not in res.terms


def test_merge_after_full_trotter_layer_matches_dense():
    """Sec. IV's Ising example merges only after a full Trotter layer (three
    symmetric sub-layers).  The layer is symmetric as a whole, so after its
    merge the representatives carry the dense orbit sums, exactly as with a
    merge after every sub-layer; in between, the set holds
    non-representative strings (more terms than the merged schedule)."""
    n = 5
    layer = W.tilted_ising_ring(n, 3, 0.3, merge="layer")
    sub = W.tilted_ising_ring(n, 3, 0.3, merge="sublayer")
    a = O.run_program(layer)
    b = O.run_program(sub)
    Od = dense.heisenberg(layer)
    coeffs = {k: v.real for k, v in dense.pauli_coefficients(Od, n).items()}
    want = orbit_sums(coeffs, n, "Zn")
    assert_terms_match(a.terms, {k: v for k, v in want.items() if abs(v) > 1e-13})
    assert_terms_match(a.terms, b.terms)
    e = dense.expectation(Od, layer.bloch, n)
    assert abs(a.expectation - e) < 1e-12 and abs(b.expectation - e) < 1e-12
    # merges happen at sub-layers 3, 6, 9 (Heisenberg order), where both
    # schedules hold the same representatives; before them the deferred
    # schedule holds at least as many strings
    assert a.sizes[2::3] == b.sizes[2::3]
    assert all(x >= y for x, y in zip(a.sizes, b.sizes))
    assert any(x > y for x, y in zip(a.sizes, b.sizes))


def test_total_spin_is_invariant_under_isotropic_layers():
    """S^2 commutes with every exp(-i theta sum_{i<j} P_i P_j): at p = 0 and
    without truncation the merged set returns to {I, XX, YY, ZZ} with the
    initial coefficients (others vanish)."""
    n = 6
    prog = W.heisenberg_all_to_all(n, 2, 0.37, obs=W.total_spin_squared(n),
                                   bloch=W.PLUS_STATE)
    res = O.run_program(prog)
    big = {k: v for k, v in res.terms.items() if abs(v) > 1e-12}
    want = {(0, 0): 0.75 * n}
    for kind in "XYZ":
        want[O.canon(n, "Sn", *W.two_site(kind, 0, 1))] = n * (n - 1) / 4
    assert set(big) == set(want)
    for k, v in want.items():
        assert abs(big[k] - v) < 1e-12 * n * n
    assert abs(res.expectation - n * (n + 2) / 4) < 1e-11


@pytest.mark.parametrize("group", ["Zn", "none"])
def test_noise_matches_density_matrix(group):
    n = 4
    prog = small_ring(n, steps=2, theta=0.4, delta=0.7, obs=W.sum_ring_pairs(n, "Z"),
                      bloch=W.random_bloch(21), p=0.07)
    res = O.run_program(prog, group=group)
    assert abs(res.expectation - dense.noisy_expectation(prog)) < 1e-12


def test_noise_matches_density_matrix_sn():
    n = 4
    prog = W.heisenberg_all_to_all(n, 1, 0.3, obs=W.sum_single(n, "Z"),
                                   bloch=W.random_bloch(4), p=0.05)
    res = O.run_program(prog)
    assert abs(res.expectation - dense.noisy_expectation(prog)) < 1e-12


def test_truncation_rules():
    n = 5
    o = O.Oracle(n, "none")
    o.add(*W.from_letters("XIIII"), 1e-3)        # exactly eps: kept
    o.add(*W.from_letters("IXIII"), 0.999e-3)    # below eps: dropped
    o.add(*W.from_letters("XXXII"), 1.0)         # weight 3 > 2: dropped
    o.add(*W.from_letters("XXIII"), -1.0)        # weight 2: kept
    o.truncate(1e-3, 2)
    assert set(o.as_dict()) == {W.from_letters("XIIII"), W.from_letters("XXIII")}


def test_work_counters():
    """propagated = sum over gates of the live terms; merged = records
    entering every merge (each anticommuting term makes two records)."""
    n = 4
    o = O.Oracle(n, "none")
    o.add(*W.from_letters("ZIII"), 1.0)
    o.add(*W.from_letters("IZII"), 1.0)
    o.apply_gate(*W.from_letters("XXII"), 0.3, 0.0, -1)   # both anticommute
    assert o.counters() == (2, 4)
    assert o.size() == 4
    o.apply_gate(*W.from_letters("IIZZ"), 0.3, 0.0, -1)   # all commute
    assert o.counters() == (6, 8)


def test_orbit_sum_is_exactly_rounded():
    """The merge adds an orbit's coefficients exactly and rounds once, so the
    result is math.fsum's (the correctly rounded sum), in any order."""
    rng = random.Random(17)
    for _ in range(300):
        k = rng.randint(0, 40)
        g = [rng.gauss(0, 1) * 10.0 ** rng.uniform(-12, 12) for _ in range(k)]
        g += [-v for v in g[: k // 3]]
        rng.shuffle(g)
        assert O.exact_sum(g) == math.fsum(g)
    assert O.exact_sum([1e16, 1.0, -1e16]) == 1.0
    # through the merge itself: three translates of one string, cancelling
    n = 4
    o = O.Oracle(n, "Zn")
    for s, c in (("XIII", 1e16), ("IXII", 1.0), ("IIXI", -1e16)):
        o.add(*W.from_letters(s), c)
    o.merge()
    assert o.as_dict() == {W.from_letters("XIII"): 1.0}


@pytest.mark.parametrize("n,group", [(5, "Zn"), (6, "Zn"), (5, "Sn"), (6, "Dn"), (4, "none")])
def test_merge_of_raw_records_against_brute_force(n, group):
    """Algorithm 1 step 1 on raw rows with many repeats: each representative
    is the orbit's lowest integer (brute force over the group with the
    independent encoding) and its coefficient the correctly rounded sum of
    every row of the orbit (math.fsum), repeated rows as separate addends."""
    rng = random.Random(23 + n)
    base = [random_string(rng, n) for _ in range(12)]
    rows = []
    for _ in range(400):
        s = rng.choice(base)
        if group in ("Zn", "Dn"):
            s = rotate_letters(s, rng.randrange(n))
            if group == "Dn" and rng.random() < 0.5:
                s = s[::-1]
        elif group == "Sn":
            s = "".join(rng.sample(s, n))
        rows.append((s, rng.gauss(0, 1) * 10.0 ** rng.uniform(-8, 8)))
    rows += [(rows[0][0], -rows[0][1]), (rows[1][0], 1e16), (rows[1][0], -1e16)]

    def images(s):
        if group == "Zn":
            return [rotate_letters(s, j) for j in range(n)]
        if group == "Dn":
            return [rotate_letters(t, j) for t in (s, s[::-1]) for j in range(n)]
        if group == "Sn":
            return ["".join(p) for p in itertools.permutations(s)]
        return [s]

    want = {}
    for s, c in rows:
        rep = min(images(s), key=lambda t: sum(DIGIT[ch] * 4 ** q for q, ch in enumerate(t)))
        want.setdefault(W.from_letters(rep), []).append(c)
    want = {k: math.fsum(v) for k, v in want.items()}
    x = np.array([W.from_letters(s)[0] for s, _ in rows], dtype=np.uint64)
    z = np.array([W.from_letters(s)[1] for s, _ in rows], dtype=np.uint64)
    got = O.merge_records(n, group, x, z, [c for _, c in rows])
    assert got == want


# ----------------------------------------------------------------------------
# Dihedral group D_n (translations and the reflection of the ring)
# ----------------------------------------------------------------------------
def bracelets(n, k=4):
    """Burnside count of k-colourings of an n-cycle up to rotation and
    reflection (the orbit count of D_n on n-qubit Pauli strings)."""
    neck = sum(k ** math.gcd(j, n) for j in range(1, n + 1))       # n * necklaces
    refl = (n // 2) * (k ** (n // 2 + 1) + k ** (n // 2)) if n % 2 == 0 else n * k ** ((n + 1) // 2)
    return (neck + refl) // (2 * n)


def test_bracelet_formula_small_values():
    # the formula against plain enumeration of colourings (no Pauli code)
    for n in range(1, 7):
        seen = set()
        for s in itertools.product(range(4), repeat=n):
            rots = [s[j:] + s[:j] for j in range(n)]
            seen.add(min(rots + [tuple(reversed(r)) for r in rots]))
        assert len(seen) == bracelets(n)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8])
def test_dihedral_representative_count(n):
    reps = set()
    for s in itertools.product("IXYZ", repeat=n):
        reps.add(O.canon(n, "Dn", *W.from_letters("".join(s))))
    assert len(reps) == bracelets(n)


@pytest.mark.parametrize("n", [4, 7, 16, 31, 32, 33, 48, 64])
def test_dihedral_representative_is_orbit_minimum(n):
    rng = random.Random(100 + n)
    for trial in range(30):
        s = random_string(rng, n, None if trial % 2 else rng.randint(0, min(n, 9)))
        rx, rz = O.canon(n, "Dn", *W.from_letters(s))
        # the orbit written out with letters: rotations of s and of s reversed
        orbit = [rotate_letters(s, j) for j in range(n)] + \
                [rotate_letters(s[::-1], j) for j in range(n)]
        best = min(orbit, key=lambda t: int_value(*W.from_letters(t), n))
        assert W.to_letters(rx, rz, n) == best
        assert O.canon(n, "Dn", rx, rz) == (rx, rz)                  # idempotent
        g = orbit[rng.randrange(2 * n)]
        assert O.canon(n, "Dn", *W.from_letters(g)) == (rx, rz)      # invariant
        # never above the translation representative
        tx, tz = O.canon(n, "Zn", *W.from_letters(s))
        assert int_value(rx, rz, n) <= int_value(tx, tz, n)


@pytest.mark.parametrize("n,obs", [(4, "Z"), (5, "XX")])
def test_dihedral_pp_matches_dense_orbit_sums(n, obs):
    ob = W.sum_single(n, "Z") if obs == "Z" else W.sum_ring_pairs(n, "X")
    prog = small_ring(n, obs=ob, bloch=W.random_bloch(2 * n))
    res = O.run_program(prog, group="Dn")
    Od = dense.heisenberg(prog)
    coeffs = {k: v.real for k, v in dense.pauli_coefficients(Od, n).items()}
    want = orbit_sums(coeffs, n, "Dn")
    assert_terms_match(res.terms, {k: v for k, v in want.items() if abs(v) > 1e-13})
    assert abs(res.expectation - dense.expectation(Od, prog.bloch, n)) < 1e-12


def test_theorem1_dihedral_equals_plain_and_translation():
    """The ring XXZ layers are reflection-symmetric, so D_n merging keeps the
    plain expectation (Theorem 1) with at most as many representatives as
    Z_n merging, and at least ceil(N / 2n)."""
    for n, steps in ((9, 3), (10, 2)):
        prog = W.xxz_ring(n, steps, 0.21, 1.3, obs=W.sum_ring_pairs(n, "X"),
                          bloch=W.random_bloch(n))
        d = O.run_program(prog, group="Dn", keep_terms=False)
        z = O.run_program(prog, group="Zn", keep_terms=False)
        b = O.run_program(prog, group="none", keep_terms=False)
        assert abs(d.expectation - b.expectation) < 1e-12 * max(1, abs(b.expectation))
        assert math.ceil(b.sizes[-1] / (2 * n)) <= d.sizes[-1] <= z.sizes[-1] <= b.sizes[-1]


# ----------------------------------------------------------------------------
# 2D translations Z_lx x Z_ly of a torus
# ----------------------------------------------------------------------------
def torus_shift(s, a, b, lx, ly):
    """Letters: site (x, y) of the result carries site (x+a, y+b) of s."""
    return "".join(s[(x + a) % lx + lx * ((y + b) % ly)] for y in range(ly) for x in range(lx))


def torus_orbit_count(lx, ly, k=4):
    """Burnside: average over the lx*ly translations of k^(number of cycles
    of the site permutation), the cycles found by following the map."""
    n = lx * ly
    total = 0
    for a in range(lx):
        for b in range(ly):
            seen, cycles = set(), 0
            for q in range(n):
                if q in seen:
                    continue
                cycles += 1
                while q not in seen:
                    seen.add(q)
                    q = (q % lx + a) % lx + lx * ((q // lx + b) % ly)
            total += k ** cycles
    return total // n


@pytest.mark.parametrize("lx,ly", [(2, 2), (2, 3), (3, 3), (2, 4), (4, 2)])
def test_torus_representative_count(lx, ly):
    n = lx * ly
    reps = set()
    for s in itertools.product("IXYZ", repeat=n):
        reps.add(O.canon(n, "T2", *W.from_letters("".join(s)), lx=lx))
    assert len(reps) == torus_orbit_count(lx, ly)


@pytest.mark.parametrize("lx,ly", [(3, 4), (4, 4), (6, 6), (8, 8)])
def test_torus_representative_is_orbit_minimum(lx, ly):
    n = lx * ly
    rng = random.Random(lx * 100 + ly)
    for trial in range(20):
        s = random_string(rng, n, None if trial % 2 else rng.randint(0, min(n, 9)))
        rx, rz = O.canon(n, "T2", *W.from_letters(s), lx=lx)
        orbit = [torus_shift(s, a, b, lx, ly) for a in range(lx) for b in range(ly)]
        best = min(orbit, key=lambda t: int_value(*W.from_letters(t), n))
        assert W.to_letters(rx, rz, n) == best
        assert O.canon(n, "T2", rx, rz, lx=lx) == (rx, rz)
        g = orbit[rng.randrange(len(orbit))]
        assert O.canon(n, "T2", *W.from_letters(g), lx=lx) == (rx, rz)


def test_torus_pp_matches_dense_orbit_sums():
    prog = W.power_law_xxz_torus(2, 3, 1, 0.15, obs=W.sum_single(6, "Z"),
                                 bloch=W.random_bloch(6))
    res = O.run_program(prog)
    Od = dense.heisenberg(prog)
    coeffs = {k: v.real for k, v in dense.pauli_coefficients(Od, 6).items()}
    sums = {}
    for (x, z), c in coeffs.items():
        r = O.canon(6, "T2", x, z, lx=2)
        sums[r] = sums.get(r, 0.0) + c
    assert_terms_match(res.terms, {k: v for k, v in sums.items() if abs(v) > 1e-13})
    assert abs(res.expectation - dense.expectation(Od, prog.bloch, 6)) < 1e-12


def test_theorem1_torus_equals_plain():
    prog = W.power_law_xxz_torus(3, 3, 1, 0.1, bloch=W.random_bloch(9))
    t = O.run_program(prog, keep_terms=False)
    b = O.run_program(prog, group="none", keep_terms=False)
    assert abs(t.expectation - b.expectation) < 1e-12 * max(1, abs(b.expectation))
    assert math.ceil(b.sizes[-1] / 9) <= t.sizes[-1] <= b.sizes[-1]


# ----------------------------------------------------------------------------
# Any finite group of qubit permutations, given by its element list
# ----------------------------------------------------------------------------
def burnside_count(perms, k=4):
    """(1/|G|) sum_g k^(cycles of g), cycles found by following each map."""
    total = 0
    for p in perms:
        seen, cycles = set(), 0
        for q in range(len(p)):
            if q in seen:
                continue
            cycles += 1
            while q not in seen:
                seen.add(q)
                q = p[q]
        total += k ** cycles
    assert total % len(perms) == 0
    return total // len(perms)


def klein_four():
    return [[0, 1, 2, 3], [1, 0, 3, 2], [2, 3, 0, 1], [3, 2, 1, 0]]


def cyclic_6_on_5():
    """The cyclic group generated by (0 1 2)(3 4), order 6."""
    g = [1, 2, 0, 4, 3]
    els, cur = [], list(range(5))
    for _ in range(6):
        els.append(cur)
        cur = [cur[g[q]] for q in range(5)]
    return els


@pytest.mark.parametrize("name", ["klein4", "c6on5", "s3", "d5", "torus2x3"])
def test_explicit_group_representative_count(name):
    perms, n = {"klein4": (klein_four(), 4), "c6on5": (cyclic_6_on_5(), 5),
                "s3": (W.elements_symmetric(3), 3), "d5": (W.elements_dihedral(5), 5),
                "torus2x3": (W.elements_torus(2, 3), 6)}[name]
    reps = set()
    for s in itertools.product("IXYZ", repeat=n):
        reps.add(O.canon(n, "G", *W.from_letters("".join(s)), perms=perms))
    assert len(reps) == burnside_count(perms)


def test_explicit_group_agrees_with_the_named_groups():
    rng = random.Random(3)
    for n in (5, 12, 32, 40):
        for _ in range(10):
            s = random_string(rng, n)
            xz = W.from_letters(s)
            assert O.canon(n, "G", *xz, perms=W.elements_ring(n)) == O.canon(n, "Zn", *xz)
            assert O.canon(n, "G", *xz, perms=W.elements_dihedral(n)) == O.canon(n, "Dn", *xz)
    for lx, ly in ((3, 4), (6, 6)):
        for _ in range(10):
            s = random_string(rng, lx * ly)
            xz = W.from_letters(s)
            assert O.canon(lx * ly, "G", *xz, perms=W.elements_torus(lx, ly)) == \
                O.canon(lx * ly, "T2", *xz, lx=lx)
    for n in (3, 5):
        for s in itertools.islice(itertools.product("IXYZ", repeat=n), 0, None, 7):
            xz = W.from_letters("".join(s))
            assert O.canon(n, "G", *xz, perms=W.elements_symmetric(n)) == O.canon(n, "Sn", *xz)


def test_theorem1_explicit_group():
    """The ring circuit merged under D_n given as a list: the same sets and
    expectation as D_n, and the plain expectation (Theorem 1)."""
    prog = W.xxz_ring(9, 2, 0.21, 1.3, obs=W.sum_ring_pairs(9, "X"), bloch=W.random_bloch(9))
    g = O.run_program(W.with_explicit_group(prog, W.elements_dihedral(9)))
    d = O.run_program(prog, group="Dn")
    b = O.run_program(prog, group="none", keep_terms=False)
    assert g.terms == d.terms and g.expectation == d.expectation
    assert abs(g.expectation - b.expectation) < 1e-12 * max(1, abs(b.expectation))
