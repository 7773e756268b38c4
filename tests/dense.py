"""Dense 2^n reference for the oracle's pins (test infrastructure).

Builds Pauli strings as explicit matrices (Kronecker products of the 2x2
Pauli matrices), the circuit unitary from the gates exp(-i theta/2 P), and
evaluates U^dag O U, its Pauli coefficients Tr[P U^dag O U] / 2^n, product
state expectations and a density-matrix simulation with depolarising noise.
It shares nothing with the oracle or the HIP library: every quantity is
computed from the matrices themselves.
"""
from __future__ import annotations

import numpy as np

SIGMA = {
    "I": np.eye(2, dtype=complex),
    "X": np.array([[0, 1], [1, 0]], dtype=complex),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=complex),
    "Z": np.array([[1, 0], [0, -1]], dtype=complex),
}


def letter(x: int, z: int, q: int) -> str:
    bx, bz = (x >> q) & 1, (z >> q) & 1
    return {(0, 0): "I", (1, 0): "X", (1, 1): "Y", (0, 1): "Z"}[(bx, bz)]


def pauli_matrix(x: int, z: int, n: int) -> np.ndarray:
    """Qubit q is bit q of the computational-basis index (qubit n-1 is the
    leftmost Kronecker factor)."""
    m = np.ones((1, 1), dtype=complex)
    for q in reversed(range(n)):
        m = np.kron(m, SIGMA[letter(x, z, q)])
    return m


def rotation(x: int, z: int, theta: float, n: int) -> np.ndarray:
    P = pauli_matrix(x, z, n)
    return np.cos(theta / 2) * np.eye(2 ** n) - 1j * np.sin(theta / 2) * P


def circuit_unitary(prog) -> np.ndarray:
    """U = V_last ... V_first for the time-ordered gates of `prog`."""
    n = prog.n
    U = np.eye(2 ** n, dtype=complex)
    for sub in prog.sublayers:
        for g in sub.gates:
            U = rotation(g.x, g.z, g.theta, n) @ U
    return U


def observable(prog) -> np.ndarray:
    O = np.zeros((2 ** prog.n, 2 ** prog.n), dtype=complex)
    for x, z, c in prog.obs:
        O += c * pauli_matrix(x, z, prog.n)
    return O


def heisenberg(prog) -> np.ndarray:
    U = circuit_unitary(prog)
    return U.conj().T @ observable(prog) @ U


def pauli_phase_perm(x: int, z: int, n: int):
    """P = i^{|x&z|} X^x Z^z, so P|k> = i^{|x&z|} (-1)^{|z&k|} |k ^ x>.
    Returns the column phases of P (entry P[k^x, k]); checked against
    pauli_matrix in the tests."""
    k = np.arange(2 ** n)
    par = np.zeros(2 ** n, dtype=np.int64)
    zk = z & k
    for q in range(n):
        par ^= (zk >> q) & 1
    return (1j ** bin(x & z).count("1")) * (1.0 - 2.0 * par)


def pauli_coefficients(O: np.ndarray, n: int) -> dict:
    """{(x, z): Tr[P O] / 2^n} over all 4^n strings (unnormalised basis)."""
    out = {}
    N = 2 ** n
    k = np.arange(N)
    for x in range(N):
        Ox = O[k, k ^ x]                       # O[k, k^x]
        for z in range(N):
            ph = pauli_phase_perm(x, z, n)     # P[k^x, k]
            out[(x, z)] = np.sum(ph * Ox) / N
    return out


def product_state(bloch, n: int) -> np.ndarray:
    """|psi>^{(x)n} with the single-qubit Bloch vector `bloch`."""
    bx, by, bz = bloch
    th = np.arccos(np.clip(bz, -1.0, 1.0))
    ph = np.arctan2(by, bx)
    psi = np.array([np.cos(th / 2), np.exp(1j * ph) * np.sin(th / 2)])
    v = np.ones(1, dtype=complex)
    for _ in range(n):
        v = np.kron(v, psi)   # all factors equal: the ordering is immaterial
    return v


def expectation(O: np.ndarray, bloch, n: int) -> float:
    v = product_state(bloch, n)
    return float(np.real(v.conj() @ O @ v))


def noisy_expectation(prog) -> float:
    """Density-matrix evolution: every sub-layer's gates, then on every qubit
    the depolarising channel rho -> (1-p) rho + p Tr_q(rho) (x) I/2."""
    n = prog.n
    v = product_state(prog.bloch, n)
    rho = np.outer(v, v.conj())
    for sub in prog.sublayers:
        for g in sub.gates:
            V = rotation(g.x, g.z, g.theta, n)
            rho = V @ rho @ V.conj().T
        if sub.p > 0:
            for q in range(n):
                rho = depolarise(rho, q, n, sub.p)
    return float(np.real(np.trace(observable(prog) @ rho)))


def depolarise(rho: np.ndarray, q: int, n: int, p: float) -> np.ndarray:
    # (1-p) rho + (p/4) sum_{P in I,X,Y,Z on qubit q} P rho P
    #   = (1-p) rho + p Tr_q(rho) (x) I/2
    acc = np.zeros_like(rho)
    for L in "IXYZ":
        bx = 1 if L in "XY" else 0
        bz = 1 if L in "YZ" else 0
        P = pauli_matrix(bx << q, bz << q, n)
        acc += P @ rho @ P
    return (1 - p) * rho + (p / 4) * acc
