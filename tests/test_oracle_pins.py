"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints (tests/golden), closed forms, invariants, an independent
brute-force definition, or textbook identities."""
import math

import numpy as np
import pytest

import oracle
from oracle import bruteforce as bf
from supremacy_inputs import (Circuit, Gate, drop_trailing_cz_layer, haar_unitary,
                              mirror_circuit, random_state, supremacy_circuit)

from conftest import read_golden


# ------------------------------------------------------------------ printed values
def test_x0_worked_example():
    """Sec. 2: X on bit-index 0 maps (a0, a1, a2, a3) -> (a1, a0, a3, a2)."""
    rows = read_golden("x0_example.txt")
    psi = np.array([1 + 2j, 3 - 1j, -0.5 + 0.25j, 2j])
    out = oracle.apply_named(psi.copy(), "X", 0)
    out_bf = bf.run(Circuit(2, [Gate("X", (0,))]), psi)
    for a, b in rows:
        assert out[int(b)] == psi[int(a)]
        assert out_bf[int(b)] == psi[int(a)]


def test_gate_matrices_as_printed():
    """The oracle's and the brute force's matrices equal the printed ones."""
    for row in read_golden("gate_matrices_sec2.txt"):
        name, vals = row[0], np.array(row[1:], dtype=float)
        z = vals[0::2] + 1j * vals[1::2]
        if name == "CZDIAG":
            np.testing.assert_array_equal(np.diag(bf.CZ4), z)
            continue
        m = z.reshape(2, 2)
        np.testing.assert_allclose(oracle.gate_matrix(name), m, rtol=0, atol=2.3e-16)  # 1/sqrt2 within 2 ulp
        np.testing.assert_allclose(bf.MATS[name], m, rtol=0, atol=2.3e-16)


def test_gate_algebra():
    """H^2 = I, T^8 = I, (X^1/2)^2 = X, (Y^1/2)^2 = Y, CZ^2 = I, U U^+ = I,
    and each dagger gate inverts its gate."""
    g = {nm: oracle.gate_matrix(nm) for nm in
         ("H", "T", "SX", "SY", "X", "Y", "Z", "TDG", "SXDG", "SYDG")}
    I2 = np.eye(2)
    tol = 1e-15
    np.testing.assert_allclose(g["H"] @ g["H"], I2, atol=tol)
    np.testing.assert_allclose(np.linalg.matrix_power(g["T"], 8), I2, atol=tol)
    np.testing.assert_allclose(np.linalg.matrix_power(g["T"], 4), g["Z"], atol=tol)
    np.testing.assert_allclose(g["SX"] @ g["SX"], g["X"], atol=tol)
    np.testing.assert_allclose(g["SY"] @ g["SY"], g["Y"], atol=tol)
    for nm, m in g.items():
        np.testing.assert_allclose(m @ m.conj().T, I2, atol=tol)
    for nm in ("T", "SX", "SY"):
        np.testing.assert_allclose(g[nm + "DG"] @ g[nm], I2, atol=tol)
    np.testing.assert_array_equal(bf.CZ4 @ bf.CZ4, np.eye(4))


# ------------------------------------------------------------------ brute force
def _random_circuit(n, n_gates, seed, dense_k=(2, 3)):
    rng = np.random.default_rng(seed)
    names = ["H", "T", "SX", "SY", "X", "Y", "Z", "TDG", "SXDG", "SYDG"]
    gates = []
    for i in range(n_gates):
        r = rng.random()
        if r < 0.55:
            gates.append(Gate(names[rng.integers(len(names))], (int(rng.integers(n)),)))
        elif r < 0.85 and n >= 2:
            a, b = rng.choice(n, 2, replace=False)
            gates.append(Gate("CZ", (int(a), int(b))))
        elif r >= 0.85:
            k = int(rng.choice(dense_k))
            qs = tuple(int(q) for q in rng.choice(n, k, replace=False))
            gates.append(Gate("U", qs, haar_unitary(k, seed * 1000 + i)))
    return Circuit(n, gates)


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (3, 2), (5, 3), (7, 4), (9, 5), (10, 6)])
def test_oracle_matches_bruteforce(n, seed):
    circ = _random_circuit(n, 40, seed, dense_k=tuple(k for k in (2, 3) if k <= n) or (1,))
    psi0 = random_state(n, seed)
    ref = bf.run(circ, psi0)
    got = oracle.apply(psi0.copy(), circ)
    assert np.max(np.abs(got - ref)) <= 1e-13


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_dense_gate_matches_bruteforce(k):
    n = 8
    rng = np.random.default_rng(k)
    qs = tuple(int(q) for q in rng.choice(n, k, replace=False))
    u = haar_unitary(k, 77 + k)
    psi0 = random_state(n, k)
    ref = bf.embed_k(u, qs, n) @ psi0
    got = oracle.apply_dense(psi0.copy(), qs, u)
    assert np.max(np.abs(got - ref)) <= 1e-13


def test_dense_bit_order_is_kronecker_of_1q():
    """A two-qubit matrix U1 (x) U0 on qubits (a, b) (bit 0 of the index <-> a)
    equals U0 on a followed by U1 on b (textbook Kronecker identity)."""
    n = 6
    u0, u1 = haar_unitary(1, 3), haar_unitary(1, 4)
    psi0 = random_state(n, 9)
    a, b = 4, 1
    got = oracle.apply_dense(psi0.copy(), (a, b), np.kron(u1, u0))
    ref = psi0.copy()
    oracle.apply_dense(ref, (a,), u0)
    oracle.apply_dense(ref, (b,), u1)
    assert np.max(np.abs(got - ref)) <= 1e-14
    # the same through the 1q path of the oracle
    ref2 = psi0.copy()
    oracle.lib().oracle_apply_1q(oracle._dptr(ref2), n, a, oracle._dptr(np.ascontiguousarray(u0)))
    oracle.lib().oracle_apply_1q(oracle._dptr(ref2), n, b, oracle._dptr(np.ascontiguousarray(u1)))
    assert np.max(np.abs(got - ref2)) <= 1e-14


def test_dense_qubit_order_permutation():
    """Listing the target qubits in another order with the matrix's index bits
    permuted the same way gives the same result."""
    n, k = 7, 3
    u = haar_unitary(k, 5)
    qs = (5, 0, 3)
    perm = (2, 0, 1)  # new bit j <- old bit perm[j]
    d = 2 ** k
    P = np.zeros((d, d))
    for x in range(d):
        y = 0
        for j in range(k):
            y |= ((x >> perm[j]) & 1) << j
        P[y, x] = 1
    u2 = P @ u @ P.T
    qs2 = tuple(qs[perm[j]] for j in range(k))
    psi0 = random_state(n, 11)
    a = oracle.apply_dense(psi0.copy(), qs, u)
    b = oracle.apply_dense(psi0.copy(), qs2, u2)
    assert np.max(np.abs(a - b)) <= 1e-14


def test_cluster_matrix_is_product():
    """The oracle's cluster matrix equals the brute-force product of the
    gates' embedded operators, and is unitary."""
    for k, seed in [(1, 0), (2, 1), (3, 2), (4, 3), (5, 4), (6, 5)]:
        circ = _random_circuit(k, 25, seed, dense_k=tuple(x for x in (2, 3) if x <= k) or (1,))
        m = oracle.cluster_matrix(k, [(g.name, g.qubits, g.mat) for g in circ.gates])
        ref = bf.circuit_unitary(circ)
        assert np.max(np.abs(m - ref)) <= 1e-13
        assert np.max(np.abs(m @ m.conj().T - np.eye(2 ** k))) <= 1e-13


# ------------------------------------------------------------------ closed forms
@pytest.mark.parametrize("n", [1, 4, 12, 20])
def test_hadamard_layer_uniform(n):
    """H^{(x)n}|0> = 2^{-n/2} (1, ..., 1)."""
    circ = Circuit(n, [Gate("H", (q,)) for q in range(n)])
    psi = oracle.run(circ)
    target = 2.0 ** (-n / 2)
    assert np.max(np.abs(psi - target)) <= 1e-15 * max(1, n) * target + 1e-300


def test_norm_and_mirror_20q():
    """Unit norm after a 20-qubit depth-25 circuit; C then C^+ returns |0>."""
    circ = supremacy_circuit(4, 5, 25, seed=0)
    psi = oracle.run(circ)
    norm, _, _ = oracle.stats(psi)
    assert abs(norm - 1.0) <= 1e-12
    back = oracle.run(mirror_circuit(circ))
    assert abs(abs(back[0]) ** 2 - 1.0) <= 1e-12
    assert np.max(np.abs(back[1:])) <= 1e-12


def test_final_cz_layer_leaves_probabilities():
    """Sec. 3.6: the final CZ layer changes phases only."""
    circ = supremacy_circuit(4, 4, 17, seed=3)
    a = oracle.run(circ)
    b = oracle.run(drop_trailing_cz_layer(circ))
    assert np.max(np.abs(np.abs(a) ** 2 - np.abs(b) ** 2)) <= 1e-15
    assert np.max(np.abs(a - b)) > 1e-3  # the phases did change


def test_drop_trailing_diagonal():
    """Sec. 3.6 generalised: diagonal gates that only meet diagonal gates
    afterwards commute to the end and change phases only. A hand-worked case
    (T on qubit 0 commutes past the CZ; the CZ is followed by H on qubit 1),
    then a supremacy circuit: the whole final CZ layer goes, and the
    probabilities (brute force and oracle) do not change."""
    small = Circuit(2, [Gate("H", (0,)), Gate("T", (0,)), Gate("CZ", (0, 1)), Gate("H", (1,)),
                        Gate("T", (1,))])
    kept, dropped = oracle.drop_trailing_diagonal(small)
    assert dropped == [1, 4]
    assert [g.name for g in kept.gates] == ["H", "CZ", "H"]
    psi0 = random_state(2, 4)
    a, b = bf.run(small, psi0.copy()), bf.run(kept, psi0.copy())
    assert np.max(np.abs(np.abs(a) ** 2 - np.abs(b) ** 2)) <= 1e-15
    circ = supremacy_circuit(3, 3, 17, seed=6)
    kept, dropped = oracle.drop_trailing_diagonal(circ)
    last = max(g.cycle for g in circ.gates)
    final_cz = {i for i, g in enumerate(circ.gates) if g.cycle == last and g.name == "CZ"}
    assert final_cz and final_cz <= set(dropped)
    assert all(circ.gates[i].name in ("CZ", "T") for i in dropped)
    full, cut = oracle.run(circ), oracle.run(kept)
    assert np.max(np.abs(np.abs(full) ** 2 - np.abs(cut) ** 2)) <= 1e-15
    bfull, bcut = bf.run(circ), bf.run(kept)
    assert np.max(np.abs(np.abs(bfull) ** 2 - np.abs(bcut) ** 2)) <= 1e-15
    assert np.max(np.abs(full - cut)) > 1e-3  # phases changed: the gates really went


def test_permute_bits():
    """Relabelling bit locations: a hand-worked swap of bits 0 and 1, and the
    identity that moving the bits equals running the circuit with every qubit
    renamed to its new location (gates on other qubit indices, from |0...0>,
    which every relabelling leaves unchanged)."""
    psi = np.array([1, 2, 3, 4], np.complex128)
    np.testing.assert_array_equal(oracle.permute_bits(psi, [0, 1], [1, 0]), [1, 3, 2, 4])
    np.testing.assert_array_equal(oracle.permute_bits(psi, [1], [1]), psi)
    circ = supremacy_circuit(3, 3, 14, seed=9)
    n = circ.n
    rng = np.random.default_rng(1)
    for src_n in (2, 3, 5, 9):
        src = [int(x) for x in rng.choice(n, src_n, replace=False)]
        dst = [int(x) for x in rng.permutation(src)]
        sigma = dict(zip(src, dst))
        ren = Circuit(n, [Gate(g.name, tuple(sigma.get(q, q) for q in g.qubits), g.mat) for g in circ.gates])
        want = oracle.run(ren)
        got = oracle.permute_bits(oracle.run(circ), src, dst)
        np.testing.assert_array_equal(got, want)
        back = oracle.permute_bits(got, dst, src)
        np.testing.assert_array_equal(back, oracle.run(circ))


def test_uniform_start_equals_hadamard_layer():
    """Sec. 3.6: starting from the uniform vector replaces the cycle-0 H."""
    circ = supremacy_circuit(3, 4, 12, seed=2)
    full = oracle.run(circ)
    rest = Circuit(circ.n, [g for g in circ.gates if g.cycle != 0])
    psi = np.full(2 ** circ.n, 2.0 ** (-circ.n / 2), np.complex128)
    oracle.apply(psi, rest)
    assert np.max(np.abs(full - psi)) <= 1e-14


def test_porter_thomas_20q():
    """Deep random circuits: N sum p^2 -> 2 and S -> ln N - 1 + gamma
    (Porter-Thomas; Boixo et al. 2016)."""
    n = 20
    N = 2.0 ** n
    gamma = 0.5772156649015329
    vals = []
    for seed in range(2):
        psi = oracle.run(supremacy_circuit(4, 5, 40, seed=seed))
        norm, s2, ent = oracle.stats(psi)
        vals.append((N * s2, ent))
        assert abs(norm - 1) < 1e-12
    m2 = np.mean([v[0] for v in vals])
    ent = np.mean([v[1] for v in vals])
    assert abs(m2 - 2.0) <= 0.2
    assert abs(ent - (math.log(N) - 1 + gamma)) <= 0.05


def test_stats_closed_forms():
    """Uniform state: sum p^2 = 1/N, S = ln N; basis state: 1 and 0."""
    n = 10
    N = 2 ** n
    u = np.full(N, N ** -0.5, np.complex128)
    norm, s2, ent = oracle.stats(u)
    assert abs(norm - 1) < 1e-14 and abs(s2 - 1 / N) < 1e-17 and abs(ent - math.log(N)) < 1e-12
    e = np.zeros(N, np.complex128)
    e[5] = 1j
    norm, s2, ent = oracle.stats(e)
    assert norm == 1 and s2 == 1 and ent == 0
