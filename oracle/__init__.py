"""CPU oracle for state-vector quantum circuit simulation.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the GPU library never does, and this
package never imports the GPU library. It shares no code with it.

Two independent definitions of the same arithmetic:
  * ``qsim_oracle.c`` (loaded through ctypes): plain complex128, one gate at a
    time, in place, following the paper's Sec. 2 (gates, bit order, Kronecker
    embedding) and Sec. 3.2 (gather / mat-vec / scatter of a k-qubit gate);
  * ``bruteforce.py`` (numpy): the full 2^n x 2^n Kronecker-product operator of
    each gate for n <= 10, a second transcription of the printed matrices.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qsim_oracle.c")
_LIB = os.path.join(_HERE, "libqsim_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2 -ffp-contract=off, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE", _SRC,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_apply_1q.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp]
        L.oracle_apply_cz.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.oracle_apply_dense.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int), dp]
        L.oracle_apply_dense.restype = ctypes.c_int
        L.oracle_apply_named.argtypes = [dp, ctypes.c_int, ctypes.c_char_p, ctypes.c_int, ctypes.c_int]
        L.oracle_apply_named.restype = ctypes.c_int
        L.oracle_apply_text.argtypes = [dp, ctypes.c_int, ctypes.c_char_p]
        L.oracle_apply_text.restype = ctypes.c_long
        L.oracle_run_text.argtypes = [dp, ctypes.c_int, ctypes.c_char_p]
        L.oracle_run_text.restype = ctypes.c_long
        L.oracle_cluster_matrix.argtypes = [ctypes.c_int, ctypes.c_char_p, dp]
        L.oracle_cluster_matrix.restype = ctypes.c_long
        L.oracle_stats.argtypes = [dp, ctypes.c_int, dp, dp, dp]
        L.oracle_gate_matrix.argtypes = [ctypes.c_char_p, dp]
        L.oracle_gate_matrix.restype = ctypes.c_int
        L.oracle_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    assert a.dtype == np.complex128 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _text(circ_or_text) -> bytes:
    if isinstance(circ_or_text, (bytes, str)):
        t = circ_or_text
    else:
        from supremacy_inputs import to_text
        t = to_text(circ_or_text)
    return t.encode() if isinstance(t, str) else t


def gate_matrix(name: str) -> np.ndarray:
    out = np.zeros((2, 2), np.complex128)
    if lib().oracle_gate_matrix(name.encode(), _dptr(out)) != 0:
        raise ValueError(name)
    return out


def run(circ, n: int = None) -> np.ndarray:
    """State after the circuit, starting from |0...0> (complex128[2^n])."""
    n = circ.n if n is None else n
    psi = np.empty(2 ** n, np.complex128)
    rc = lib().oracle_run_text(_dptr(psi), n, _text(circ))
    if rc < 0:
        raise ValueError("oracle parse error at line %d" % -rc)
    return psi


def apply(psi: np.ndarray, circ, n: int = None) -> np.ndarray:
    """Apply the circuit's gates to ``psi`` in place and return it."""
    n = int(np.log2(psi.size)) if n is None else n
    rc = lib().oracle_apply_text(_dptr(psi), n, _text(circ))
    if rc < 0:
        raise ValueError("oracle parse error at line %d" % -rc)
    return psi


def apply_dense(psi: np.ndarray, qubits, u: np.ndarray) -> np.ndarray:
    n = int(np.log2(psi.size))
    q = (ctypes.c_int * len(qubits))(*qubits)
    u = np.ascontiguousarray(u, dtype=np.complex128)
    if lib().oracle_apply_dense(_dptr(psi), n, len(qubits), q, _dptr(u)) != 0:
        raise ValueError("bad dense gate")
    return psi


def apply_named(psi: np.ndarray, name: str, q0: int, q1: int = -1) -> np.ndarray:
    n = int(np.log2(psi.size))
    if lib().oracle_apply_named(_dptr(psi), n, name.encode(), q0, q1) != 0:
        raise ValueError("bad gate %s" % name)
    return psi


def cluster_matrix(k: int, gates) -> np.ndarray:
    """Matrix (2^k x 2^k) of a gate sequence on local qubits 0..k-1, column x
    = the sequence applied to basis vector e_x. ``gates`` is a list of
    (name, qubits[, matrix]) with local qubit indices."""
    from supremacy_inputs import Circuit, Gate, to_text
    gl = [Gate(g[0], tuple(g[1]), g[2] if len(g) > 2 else None) for g in gates]
    out = np.empty((2 ** k, 2 ** k), np.complex128)
    rc = lib().oracle_cluster_matrix(k, to_text(Circuit(k, gl)).encode(), _dptr(out))
    if rc < 0:
        raise ValueError("oracle parse error")
    return out


def stats(psi: np.ndarray):
    """(norm, sum p^2, entropy in nats) of the state, p_i = |a_i|^2."""
    n = int(np.log2(psi.size))
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    lib().oracle_stats(_dptr(psi), n, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    return a.value, b.value, c.value


def num_threads() -> int:
    return lib().oracle_num_threads()


def permute_bits(psi: np.ndarray, src, dst) -> np.ndarray:
    """Relabel bit locations (Sec. 3.4: qubits are moved between bit
    locations before and after a global-to-local swap): the amplitude at
    index i goes to the index whose bit dst[j] is bit src[j] of i, every
    other bit unchanged. Returns a new array."""
    n = int(np.log2(psi.size))
    assert sorted(src) == sorted(dst) and len(set(src)) == len(src)
    i = np.arange(psi.size, dtype=np.int64)
    j = i.copy()
    for s in src:
        j &= ~(np.int64(1) << s)
    for s, d in zip(src, dst):
        j |= ((i >> s) & 1) << d
    out = np.empty_like(psi)
    out[j] = psi
    return out


# Gates whose matrix is diagonal in the computational basis (Sec. 2: T and CZ
# as printed; Z, T^dagger and the phase gate diag(1, e^{i theta})).
DIAGONAL_GATES = frozenset({"T", "TDG", "Z", "CZ", "PHASE"})


def drop_trailing_diagonal(circ):
    """The circuit without its trailing diagonal gates (Sec. 3.6: the final CZ
    gates are not simulated, as they change phases and not the output
    probabilities). A diagonal gate is trailing when no non-diagonal gate
    comes after it on any of its qubits; diagonal gates commute with one
    another, so removing all of them multiplies every amplitude by a phase.
    Returns (circuit, indices of the removed gates)."""
    from supremacy_inputs import Circuit
    later_dense = set()
    drop = []
    for i in range(len(circ.gates) - 1, -1, -1):
        g = circ.gates[i]
        if g.name in DIAGONAL_GATES:
            if not any(q in later_dense for q in g.qubits):
                drop.append(i)
        else:
            later_dense.update(g.qubits)
    gone = set(drop)
    kept = [g for i, g in enumerate(circ.gates) if i not in gone]
    return Circuit(circ.n, kept, dict(circ.meta, trailing_diagonal_dropped=len(drop))), sorted(drop)
