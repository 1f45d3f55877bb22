"""The seeded circuit generator against the rules and counts the paper states
(Fig. 1 caption, Sec. 3.6, Table 1)."""
import numpy as np
import pytest

from supremacy_inputs import (SplitMix64, batch_circuit, batch_circuit_params, blocked_circuit,
                              cz_pattern, drop_trailing_cz_layer, grid_edges, haar_unitary,
                              mirror_circuit, supremacy_circuit, with_haar_layers)
from supremacy_inputs.circuits import grid_sites

from conftest import read_golden


def test_table1_gate_counts():
    """Gate counts of Table 1 (H included, final CZ layer excluded)."""
    for R, C, n, gates, *_ in read_golden("table1_counts.txt"):
        R, C, n, gates = int(R), int(C), int(n), int(gates)
        for (r, c) in ((R, C), (C, R)):
            circ = drop_trailing_cz_layer(supremacy_circuit(r, c, 25, seed=1))
            assert circ.n == n
            assert len(circ.gates) == gates


def test_every_edge_once_per_8_cycles():
    """Fig. 1 caption: every nearest-neighbour pair interacts once every 8 cycles."""
    for R, C in [(4, 5), (5, 6), (6, 6), (7, 6), (9, 5)]:
        sites = grid_sites(R, C)
        seen = []
        for w in range(8):
            seen.extend(cz_pattern(R, C, w, sites))
        assert sorted(seen) == grid_edges(R, C)
        assert len(set(seen)) == len(seen)


def test_single_qubit_gate_rules():
    """Fig. 1 caption: 1q gates only on qubits with a CZ in the previous cycle
    and none in the current; the first is T; a random pick differs from the
    previous 1q gate; cycle 0 is H on all qubits."""
    for seed in range(4):
        circ = supremacy_circuit(5, 6, 25, seed)
        by_cycle = {}
        for g in circ.gates:
            by_cycle.setdefault(g.cycle, []).append(g)
        assert [g.name for g in by_cycle[0]] == ["H"] * 30
        last = {q: "H" for q in range(30)}
        prev_cz = set()
        for t in range(1, 25):
            cz_q = {q for g in by_cycle[t] if g.name == "CZ" for q in g.qubits}
            one = [g for g in by_cycle[t] if g.name != "CZ"]
            assert {g.qubits[0] for g in one} == prev_cz - cz_q
            for g in one:
                q = g.qubits[0]
                assert g.name in ("T", "SX", "SY")
                if last[q] == "H":
                    assert g.name == "T"
                else:
                    assert g.name != last[q]
                last[q] = g.name
            used = [q for g in by_cycle[t] for q in g.qubits]
            assert len(used) == len(set(used))  # disjoint within a cycle
            prev_cz = cz_q


def test_seed_changes_only_gate_choice():
    a = supremacy_circuit(5, 6, 25, 0)
    b = supremacy_circuit(5, 6, 25, 1)
    assert [(g.qubits, g.cycle) for g in a.gates] == [(g.qubits, g.cycle) for g in b.gates]
    assert [g.name for g in a.gates] != [g.name for g in b.gates]


def test_34q_grid():
    circ = supremacy_circuit(5, 7, 25, 0, drop=[(4, 6)])
    assert circ.n == 34
    assert len(circ.gates) == 427
    assert len(drop_trailing_cz_layer(circ).gates) == 421
    assert max(q for g in circ.gates for q in g.qubits) == 33


def test_splitmix64_reference_values():
    """SplitMix64 outputs for seed 0 (Steele, Lea & Flood 2014; the same
    values as java.util.SplittableRandom's mixer)."""
    r = SplitMix64(0)
    assert r.next() == 0xE220A8397B1DCDAF
    assert r.next() == 0x6E789E6AA1B965F4
    assert r.next() == 0x06C45D188009454F


def test_batch_params_ranges():
    ns, ds = [], []
    for i in range(512):
        n, d, s = batch_circuit_params(i)
        assert 14 <= n <= 24 and 10 <= d <= 40 and s == 1000 + i
        ns.append(n)
        ds.append(d)
    assert len(set(ns)) == 11 and min(ds) == 10 and max(ds) == 40
    c = batch_circuit(3)
    assert c.n == batch_circuit_params(3)[0]


def test_blocked_and_haar_and_mirror():
    circ = blocked_circuit(12, [[0, 3, 6, 9, 11], [1, 4, 7, 10], [2, 5, 8]], 10, 4)
    for g in circ.gates:
        if g.name == "CZ":
            grp = [set(x) for x in circ.meta["groups"]]
            assert any(set(g.qubits) <= s for s in grp)
    h = with_haar_layers(supremacy_circuit(4, 5, 25, 0), 8, 5, 7)
    us = [g for g in h.gates if g.name == "U"]
    assert len(us) == 3 and all(len(set(g.qubits)) == 5 for g in us)
    for g in us:
        assert np.max(np.abs(g.mat @ g.mat.conj().T - np.eye(32))) < 1e-13
    m = mirror_circuit(h)
    assert len(m.gates) == 2 * len(h.gates)


def test_haar_unitary_moments():
    """|U_00|^2 of Haar U(d) has mean 1/d."""
    d = 4
    vals = [abs(haar_unitary(2, s)[0, 0]) ** 2 for s in range(400)]
    assert abs(np.mean(vals) - 1 / d) < 0.03
