"""Seeded synthetic workloads for symmetry-merging Pauli propagation.

This module only *describes* circuits: which Pauli rotations act in which
order, with which angles, on which observable, with which truncation and
noise parameters, measured in which symmetric product state.  It holds none
of the method's arithmetic (no Pauli products, no canonical forms, no
coefficient updates), so both the CPU oracle and the HIP path consume it.

Conventions (restated from the paper, arXiv:2512.12094):

* A Pauli string on ``n`` qubits is a pair of Python ints ``(x, z)``: bit
  ``q`` of ``x``/``z`` is the X/Z part of qubit ``q`` (symplectic form,
  Appendix E.2), so X=(1,0), Y=(1,1), Z=(0,1).
* A gate ``Gate(x, z, theta)`` is the rotation ``exp(-i theta/2 P)``.
* A circuit is a list of sub-layers in *time order*; every sub-layer is
  exactly symmetric under the program's group (Eq. (action), Sec. I).  The
  Heisenberg pass walks this list backwards (Algorithm 1, step 2).
* Observables are lists of ``(x, z, coef)`` rows of unnormalised Pauli
  operators.
* The initial state is a symmetric product state ``psi^{(x)n}`` given by
  its Bloch vector.
"""
from __future__ import annotations

import dataclasses

from dataclasses import dataclass, field
from typing import List, Tuple

import math

import numpy as np

GROUP_NONE = "none"
GROUP_ZN = "Zn"   # cyclic translation (Example: translation symmetry Z_n)
GROUP_SN = "Sn"   # qubit permutations (Example: permutation symmetry S_n)
GROUP_DN = "Dn"   # ring translations and reflection (dihedral D_n)
GROUP_T2 = "T2"   # translations of an lx x ly torus (width in meta["lx"])
GROUP_G = "G"     # any group of qubit permutations (element list in meta["perms"])


@dataclass(frozen=True)
class Gate:
    x: int
    z: int
    theta: float


@dataclass
class SubLayer:
    gates: List[Gate]
    eps: float = 0.0        # drop |c| < eps (0 = off)
    wmax: int = -1          # drop Pauli weight > wmax (<0 = off)
    p: float = 0.0          # depolarising strength per qubit for this sub-layer
    m: int = 1              # exact merge (and truncation) after every m gates
    merge: bool = True      # symmetry merge after this sub-layer (Alg. 1 step 2b);
                            # False defers it to a later sub-layer (Sec. IV merges
                            # only after a full Trotter layer)


@dataclass
class Program:
    name: str
    n: int
    group: str
    obs: List[Tuple[int, int, float]]
    sublayers: List[SubLayer]
    bloch: Tuple[float, float, float]
    meta: dict = field(default_factory=dict)

    @property
    def n_gates(self) -> int:
        return sum(len(s.gates) for s in self.sublayers)

    def with_group(self, group: str) -> "Program":
        """Same circuit, other merge group (plain PP uses GROUP_NONE)."""
        return Program(self.name + ("" if group == self.group else f"[{group}]"),
                       self.n, group, list(self.obs), self.sublayers, self.bloch,
                       dict(self.meta))


# ----------------------------------------------------------------------------
# Pauli string helpers that only *spell* strings (no algebra)
# ----------------------------------------------------------------------------
_LETTER = {"I": (0, 0), "X": (1, 0), "Y": (1, 1), "Z": (0, 1)}


def from_letters(s: str) -> Tuple[int, int]:
    """'XIZ' -> (x, z) with the first letter on qubit 0."""
    x = z = 0
    for q, ch in enumerate(s):
        bx, bz = _LETTER[ch]
        x |= bx << q
        z |= bz << q
    return x, z


def to_letters(x: int, z: int, n: int) -> str:
    out = []
    for q in range(n):
        bx, bz = (x >> q) & 1, (z >> q) & 1
        out.append("IXZY"[bx | (bz << 1)])
    return "".join(out)


def two_site(kind: str, i: int, j: int) -> Tuple[int, int]:
    m = (1 << i) | (1 << j)
    return {"X": (m, 0), "Y": (m, m), "Z": (0, m)}[kind]


def one_site(kind: str, i: int) -> Tuple[int, int]:
    m = 1 << i
    return {"X": (m, 0), "Y": (m, m), "Z": (0, m)}[kind]


def ring_sublayer(n: int, kind: str, theta: float, **kw) -> SubLayer:
    """R_{PP}(theta) on every ring bond (b, b+1 mod n), b = 0..n-1."""
    gates = [Gate(*two_site(kind, b, (b + 1) % n), theta) for b in range(n)]
    return SubLayer(gates, **kw)


def all_pairs_sublayer(n: int, kind: str, theta: float, **kw) -> SubLayer:
    """R_{PP}(theta) on every pair i<j, lexicographic."""
    gates = [Gate(*two_site(kind, i, j), theta)
             for i in range(n) for j in range(i + 1, n)]
    return SubLayer(gates, **kw)


def field_sublayer(n: int, kind: str, theta: float, **kw) -> SubLayer:
    gates = [Gate(*one_site(kind, i), theta) for i in range(n)]
    return SubLayer(gates, **kw)


def sum_single(n: int, kind: str, coef: float = 1.0):
    return [(*one_site(kind, i), coef) for i in range(n)]


def sum_ring_pairs(n: int, kind: str, coef: float = 1.0):
    return [(*two_site(kind, i, (i + 1) % n), coef) for i in range(n)]


def total_spin_squared(n: int):
    """S^2 = sum_mu (sum_i P_{mu,i}/2)^2 in unnormalised Pauli rows
    (Eq. (s2)): (3n/4) I + (1/2) sum_mu sum_{i<j} P_{mu,i} P_{mu,j}."""
    rows = [(0, 0, 0.75 * n)]
    for kind in "XYZ":
        for i in range(n):
            for j in range(i + 1, n):
                rows.append((*two_site(kind, i, j), 0.5))
    return rows


def random_bloch(seed: int) -> Tuple[float, float, float]:
    rng = np.random.default_rng(seed)
    v = rng.normal(size=3)
    v /= np.linalg.norm(v)
    return float(v[0]), float(v[1]), float(v[2])


ZERO_STATE = (0.0, 0.0, 1.0)   # |0>^n
PLUS_STATE = (1.0, 0.0, 0.0)   # |+>^n


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------
def xxz_ring(n: int, steps: int, theta: float, delta: float, *, eps=0.0,
             wmax=-1, p=0.0, obs=None, bloch=ZERO_STATE, group=GROUP_ZN,
             name="xxz_ring") -> Program:
    """Trotterised XXZ ring: each step is RXX(theta), RYY(theta),
    RZZ(delta*theta) on all ring bonds (three Z_n-symmetric sub-layers)."""
    subs = []
    for _ in range(steps):
        for kind, th in (("X", theta), ("Y", theta), ("Z", delta * theta)):
            subs.append(ring_sublayer(n, kind, th, eps=eps, wmax=wmax, p=p))
    if obs is None:
        obs = sum_single(n, "Z")
    return Program(name, n, group, obs, subs, bloch,
                   dict(steps=steps, theta=theta, delta=delta, eps=eps, wmax=wmax, p=p))


def heisenberg_all_to_all(n: int, steps: int, theta: float, *, eps=0.0, wmax=-1,
                          p=0.0, obs=None, bloch=ZERO_STATE, group=GROUP_SN,
                          name="heis_a2a") -> Program:
    """Each step: exp(-i theta sum_{i<j} P_i P_j) for P = X, Y, Z, each
    applied as C(n,2) pair rotations exp(-i theta P_i P_j) = R_PP(2 theta)."""
    # the three sub-layers repeat every step: their (read-only) gate lists
    # are built once and shared
    once = {kind: all_pairs_sublayer(n, kind, 2.0 * theta, eps=eps, wmax=wmax, p=p)
            for kind in "XYZ"}
    subs = []
    for _ in range(steps):
        for kind in "XYZ":
            subs.append(dataclasses.replace(once[kind]))
    if obs is None:
        obs = sum_single(n, "Z")
    return Program(name, n, group, obs, subs, bloch,
                   dict(steps=steps, theta=theta, eps=eps, wmax=wmax, p=p))


def tilted_ising_ring(n: int, steps: int, dt: float, gx: float = 1.4,
                      gz: float = 0.9045, merge: str = "sublayer", **kw) -> Program:
    """Trotterised tilted-field Ising ring (Sec. IV): per step the ZZ bonds,
    then the Z field, then the X field, as three Z_n-symmetric sub-layers.
    exp(-i dt Z_iZ_j) = R_ZZ(2dt); exp(-i h dt P) = R_P(2 h dt).
    merge="sublayer" merges after every sub-layer; merge="layer" only after
    a full Trotter step, as the paper's Ising example does (Sec. IV): in
    Heisenberg order a step ends with its first sub-layer in time, ZZ.
    kw (eps, wmax, p) sets every sub-layer's truncation and noise."""
    if merge not in ("sublayer", "layer"):
        raise ValueError("merge is 'sublayer' or 'layer'")
    subs = []
    for _ in range(steps):
        subs.append(ring_sublayer(n, "Z", 2.0 * dt, **kw))
        subs.append(field_sublayer(n, "Z", 2.0 * gz * dt, merge=merge == "sublayer", **kw))
        subs.append(field_sublayer(n, "X", 2.0 * gx * dt, merge=merge == "sublayer", **kw))
    mid = (n + 1) // 2 - 1   # qubit ceil(n/2) in 1-based numbering
    return Program("ising", n, GROUP_ZN, [(*one_site("Z", mid), 1.0)], subs,
                   ZERO_STATE, dict(steps=steps, dt=dt, gx=gx, gz=gz, merge=merge,
                                    eps=kw.get("eps", 0.0)))


def torus_distance(i: int, j: int, lx: int, ly: int) -> float:
    """Minimum-image Euclidean distance between sites i and j of an lx x ly
    torus (site q = x + lx*y), so every coupling is translation invariant."""
    dx = abs(i % lx - j % lx)
    dy = abs(i // lx - j // lx)
    dx, dy = min(dx, lx - dx), min(dy, ly - dy)
    return math.hypot(dx, dy)


def power_law_xxz_torus(lx: int, ly: int, steps: int, dt: float, *, delta: float = -1.8,
                        jperp: float = 1.0, alpha: float = 3.0, eps=0.0, wmax=-1,
                        obs=None, bloch=ZERO_STATE, name="xxz_torus") -> Program:
    """Trotterised power-law XXZ model on an lx x ly torus:
    H = sum_{i<j} J_ij (jperp (X_iX_j + Y_iY_j) + delta Z_iZ_j) with
    J_ij = 1 / d_ij^alpha (minimum-image distance).  Per step three
    sub-layers, XX, YY, ZZ over all pairs i<j (lexicographic); the rotation
    exp(-i dt J P_iP_j) is R_PP(2 dt J)."""
    n = lx * ly
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    J = {p: 1.0 / torus_distance(p[0], p[1], lx, ly) ** alpha for p in pairs}
    subs = []
    for _ in range(steps):
        for kind, scale in (("X", jperp), ("Y", jperp), ("Z", delta)):
            subs.append(SubLayer([Gate(*two_site(kind, i, j), 2.0 * dt * scale * J[(i, j)])
                                  for (i, j) in pairs], eps=eps, wmax=wmax))
    obs = sum_single(n, "Z") if obs is None else obs
    return Program(name, n, GROUP_T2, obs, subs, bloch,
                   dict(lx=lx, ly=ly, steps=steps, dt=dt, delta=delta, jperp=jperp,
                        alpha=alpha, eps=eps))


# ----------------------------------------------------------------------------
# Groups as explicit element lists: row g lists, for each qubit q, the qubit
# of s that qubit q of g.s carries (index permutations only).
# ----------------------------------------------------------------------------
def elements_ring(n: int) -> List[List[int]]:
    """The n translations T^j of a ring."""
    return [[(q + j) % n for q in range(n)] for j in range(n)]


def elements_dihedral(n: int) -> List[List[int]]:
    """The 2n elements T^j and T^j R (R: q -> n-1-q) of D_n."""
    rots = elements_ring(n)
    return rots + [[n - 1 - r[q] for q in range(n)] for r in rots]


def elements_torus(lx: int, ly: int) -> List[List[int]]:
    return [[(q % lx + a) % lx + lx * ((q // lx + b) % ly) for q in range(lx * ly)]
            for b in range(ly) for a in range(lx)]


def elements_symmetric(n: int) -> List[List[int]]:
    import itertools
    return [list(p) for p in itertools.permutations(range(n))]


def permute_mask(v: int, perm) -> int:
    """Relabels the qubits of a bit mask: bit q of the result is bit
    perm[q] of v."""
    return sum(((v >> src) & 1) << q for q, src in enumerate(perm))


def symmetrize(gates: List[Gate], perms) -> List[Gate]:
    """Every gate's image under every listed group element (a multiset
    closed under the group)."""
    return [Gate(permute_mask(g.x, p), permute_mask(g.z, p), g.theta)
            for g in gates for p in perms]


def with_explicit_group(prog: Program, perms) -> Program:
    """The same circuit merged under the group with element list perms."""
    meta = dict(prog.meta)
    meta["perms"] = [list(map(int, r)) for r in perms]
    return Program(prog.name + "[G]", prog.n, GROUP_G, list(prog.obs), prog.sublayers,
                   prog.bloch, meta)


def config1() -> Program:
    """Z_8 ring, RXX/RYY/RZZ(0.1) x 6 steps, O = sum Z_i, no truncation."""
    return xxz_ring(8, 6, 0.1, 1.0, name="c1_z8_ring")


def config2(group: str = GROUP_ZN, steps: int = 20) -> Program:
    """Z_32 XXZ ring, theta=0.05, Delta=1.5, 20 steps, O = sum X_i X_{i+1},
    eps=1e-4, weight <= 8, Bloch vector uniform on the sphere (seed 2512)."""
    return xxz_ring(32, steps, 0.05, 1.5, eps=1e-4, wmax=8,
                    obs=sum_ring_pairs(32, "X"), bloch=random_bloch(2512),
                    group=group, name="c2_z32_xxz")


def config3(observable: str = "sumz", steps: int = 10, n: int = 64,
            group: str = GROUP_SN) -> Program:
    """S_64 all-to-all Heisenberg, theta=0.02, 10 steps, p=1e-3, eps=1e-5.
    Primary observable sum Z_i with |0^n>; secondary S^2 with |+>^n."""
    if observable == "sumz":
        obs, bloch = sum_single(n, "Z"), ZERO_STATE
    elif observable == "s2":
        obs, bloch = total_spin_squared(n), PLUS_STATE
    else:
        raise ValueError(observable)
    return heisenberg_all_to_all(n, steps, 0.02, eps=1e-5, p=1e-3, obs=obs,
                                 bloch=bloch, group=group,
                                 name=f"c3_s{n}_heis_{observable}")


def config4(seed: int = 4, count: int = 256) -> List[Program]:
    """Batch of Z_n XXZ rings with per-instance random n, depth, angles,
    anisotropy and truncation threshold."""
    rng = np.random.default_rng(seed)
    progs = []
    for k in range(count):
        n = int(rng.choice([16, 24, 32, 48, 64]))
        steps = int(rng.integers(5, 41))
        theta = float(rng.uniform(0.01, 0.1))
        delta = float(rng.uniform(0.5, 2.0))
        eps = float(10.0 ** rng.uniform(-6, -4))
        progs.append(xxz_ring(n, steps, theta, delta, eps=eps,
                              name=f"c4_{k}_z{n}"))
    return progs


@dataclass
class Job:
    arrival: float
    program: Program


def config5(seed: int = 5, count: int = 2000, rate: float = 1.0) -> List[Job]:
    """Poisson arrivals (rate jobs/s) of a 70/30 mix of Z_n XXZ rings and
    S_n all-to-all Heisenberg jobs."""
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    for k in range(count):
        t += float(rng.exponential(1.0 / rate))
        eps = float(10.0 ** rng.uniform(-6, -3))
        if rng.random() < 0.7:
            n = int(rng.choice([16, 24, 32, 40, 48, 56, 64]))
            steps = int(rng.integers(10, 41))
            theta = float(rng.uniform(0.01, 0.1))
            delta = float(rng.uniform(0.5, 2.0))
            prog = xxz_ring(n, steps, theta, delta, eps=eps, name=f"c5_{k}_z{n}")
        else:
            n = int(rng.choice([32, 64, 96, 128]))
            steps = int(rng.integers(5, 16))
            p = float(rng.uniform(0.0, 1e-2))
            prog = heisenberg_all_to_all(n, steps, 0.02, eps=eps, p=p,
                                         name=f"c5_{k}_s{n}")
        jobs.append(Job(t, prog))
    return jobs


def merge_stress_records(log2n: int, dup: int, seed: int = 7, n: int = 32,
                         wmax: int = 8):
    """Records for the canonicalise+merge pass: random weight-<=wmax Z_n
    strings, each emitted in `dup` random cyclic rotations, with coefficients
    N(0,1) * 10^U[-4,0].  Returns numpy arrays (x, z, coef) of length 2^log2n.
    Rotations are spelled as index permutations, not Pauli algebra."""
    rng = np.random.default_rng(seed)
    N = 1 << log2n
    nbase = max(1, N // dup)
    # random support of random weight, random letters
    w = rng.integers(1, wmax + 1, size=nbase)
    pos = np.argsort(rng.random((nbase, n)), axis=1)
    letters = rng.integers(1, 4, size=(nbase, n))
    sel = np.arange(n)[None, :] < w[:, None]
    xbit = ((letters == 1) | (letters == 2)) & sel
    zbit = ((letters == 2) | (letters == 3)) & sel
    one = np.uint64(1)
    x = np.zeros(nbase, dtype=np.uint64)
    z = np.zeros(nbase, dtype=np.uint64)
    for k in range(n):
        qk = pos[:, k].astype(np.uint64)
        x |= xbit[:, k].astype(np.uint64) << qk
        z |= zbit[:, k].astype(np.uint64) << qk
    base_idx = np.repeat(np.arange(nbase), dup)[:N]
    if base_idx.size < N:
        base_idx = np.concatenate([base_idx, rng.integers(0, nbase, N - base_idx.size)])
    shift = rng.integers(0, n, size=N).astype(np.uint64)
    mask = np.uint64((1 << n) - 1) if n < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    nn = np.uint64(n)

    def rot(v):
        v = v[base_idx]
        s = shift
        out = np.where(s == 0, v, ((v << s) | (v >> (nn - s))) & mask)
        return out.astype(np.uint64)

    xs, zs = rot(x), rot(z)
    perm = rng.permutation(N)
    coef = rng.normal(size=N) * 10.0 ** rng.uniform(-4, 0, size=N)
    return xs[perm], zs[perm], coef


def words(v: int, W: int) -> List[int]:
    """Split a non-negative int into W little-endian uint64 words."""
    return [(v >> (64 * w)) & 0xFFFFFFFFFFFFFFFF for w in range(W)]


def n_words(n: int) -> int:
    return (n + 63) // 64
