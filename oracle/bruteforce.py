"""Brute-force numpy definition for small circuits (n <= 10).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Every gate becomes its full 2^n x 2^n operator:
  * a single-qubit U on qubit q is 1^{(x)(n-q-1)} (x) U (x) 1^{(x)q}, the
    Kronecker embedding of the paper's Sec. 2;
  * CZ(a, b) and dense k-qubit gates are embedded by an explicit basis
    permutation: the operator's entry <i|G|j> is U[x(i)][x(j)] when i and j
    agree on every non-target bit, and 0 otherwise (x(i) collects the target
    bits of i, bit j of x from qubit qubits[j]), as in Sec. 3.2.
The gate matrices are a second, independent transcription of the ones printed
in Sec. 2.
"""
from __future__ import annotations

import numpy as np

_r2 = 1.0 / np.sqrt(2.0)
MATS = {
    "H": _r2 * np.array([[1, 1], [1, -1]], dtype=np.complex128),
    "T": np.array([[1, 0], [0, np.exp(1j * np.pi / 4)]], dtype=np.complex128),
    "SX": 0.5 * np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]], dtype=np.complex128),
    "SY": 0.5 * np.array([[1 + 1j, -1 - 1j], [1 + 1j, 1 + 1j]], dtype=np.complex128),
    "X": np.array([[0, 1], [1, 0]], dtype=np.complex128),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    "Z": np.array([[1, 0], [0, -1]], dtype=np.complex128),
}
for _nm in ("T", "SX", "SY"):
    MATS[_nm + "DG"] = MATS[_nm].conj().T
CZ4 = np.diag([1, 1, 1, -1]).astype(np.complex128)  # basis |b1 b0>, bit 0 = first qubit


def embed_1q(u: np.ndarray, q: int, n: int) -> np.ndarray:
    """1^{(x)(n-q-1)} (x) U (x) 1^{(x)q}."""
    return np.kron(np.kron(np.eye(2 ** (n - q - 1)), u), np.eye(2 ** q))


def embed_k(u: np.ndarray, qubits, n: int) -> np.ndarray:
    """Full operator of a k-qubit matrix acting on ``qubits`` (bit j of the
    matrix index <-> qubits[j])."""
    dim = 2 ** n
    idx = np.arange(dim)
    x = np.zeros(dim, dtype=np.int64)
    rest = idx.copy()
    for j, q in enumerate(qubits):
        x |= ((idx >> q) & 1) << j
        rest &= ~(1 << q)
    same = rest[:, None] == rest[None, :]
    return np.where(same, u[x[:, None], x[None, :]], 0.0)


def gate_operator(g, n: int) -> np.ndarray:
    name, qubits = g.name, g.qubits
    if name == "CZ":
        return embed_k(CZ4, qubits, n)
    if name == "U":
        return embed_k(np.asarray(g.mat), qubits, n)
    return embed_1q(MATS[name], qubits[0], n)


def circuit_unitary(circ) -> np.ndarray:
    n = circ.n
    U = np.eye(2 ** n, dtype=np.complex128)
    for g in circ.gates:
        U = gate_operator(g, n) @ U
    return U


def run(circ, psi0: np.ndarray = None) -> np.ndarray:
    n = circ.n
    assert n <= 10, "brute force is for n <= 10"
    psi = np.zeros(2 ** n, np.complex128) if psi0 is None else psi0.astype(np.complex128).copy()
    if psi0 is None:
        psi[0] = 1.0
    for g in circ.gates:
        psi = gate_operator(g, n) @ psi
    return psi
