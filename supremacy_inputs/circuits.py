"""Boixo-style random supremacy circuits (paper, Fig. 1 caption and Sec. 3.6).

Rules, as the paper states them:
  * cycle 0 applies H to every qubit;
  * afterwards eight nearest-neighbour CZ patterns repeat cyclically, so that
    every edge of the 2D grid is used once every 8 cycles;
  * a qubit that had a CZ in the previous cycle but has none in the current one
    receives a random single-qubit gate from {T, X^1/2, Y^1/2};
  * the first such gate on each qubit is T, and a random choice always differs
    from the previous single-qubit gate on that qubit.

The drawing of the 8 patterns (Fig. 1) is not in the text, so the pattern
family used here is our own reading: four horizontal and four vertical
matchings split by column and row parity, in the fixed order
``H00, H11, V00, H10, V11, H01, V10, V01``. With H counted and the final CZ
layer excluded it gives exactly the gate counts of Table 1 (369, 447, 528 and
569 for the 6x5, 6x6, 7x6 and 9x5 grids).

Qubit numbering: a grid of R rows and C columns, qubit q = r*C + c.
Random choices come from SplitMix64 (Steele, Lea & Flood, 2014), one draw per
random (non-forced) single-qubit gate, in (cycle, qubit) order.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

# Gate names. "U" is a dense k-qubit gate whose matrix travels with it.
GATE_NAMES = ("H", "T", "SX", "SY", "X", "Y", "Z", "CZ", "TDG", "SXDG", "SYDG", "U")
# Name of the inverse of each named gate (the matrices live with the consumers).
DAGGER = {"H": "H", "T": "TDG", "SX": "SXDG", "SY": "SYDG", "X": "X", "Y": "Y",
          "Z": "Z", "CZ": "CZ", "TDG": "T", "SXDG": "SX", "SYDG": "SY"}

_MASK64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 generator (Steele, Lea & Flood, OOPSLA 2014)."""

    def __init__(self, seed: int):
        self.state = seed & _MASK64

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        return z ^ (z >> 31)

    def below(self, m: int) -> int:
        """Uniform integer in [0, m) by the multiply-shift map of the top bits."""
        return (self.next() * m) >> 64


@dataclass(frozen=True)
class Gate:
    name: str
    qubits: Tuple[int, ...]
    mat: Optional[np.ndarray] = None  # only for "U": (2^k, 2^k) complex128, bit j <-> qubits[j]
    cycle: int = -1

    @property
    def k(self) -> int:
        return len(self.qubits)


@dataclass
class Circuit:
    n: int
    gates: List[Gate]
    meta: dict = field(default_factory=dict)

    def counts(self):
        out = {}
        for g in self.gates:
            out[g.name] = out.get(g.name, 0) + 1
        return out


# ---------------------------------------------------------------- grid + patterns
def grid_sites(R: int, C: int, drop: Sequence[Tuple[int, int]] = ()) -> dict:
    """Map grid site (r, c) -> qubit index; dropped sites are removed and the
    remaining sites keep row-major order (q = r*C + c when nothing is dropped
    before them)."""
    dropped = set(drop)
    sites = {}
    q = 0
    for r in range(R):
        for c in range(C):
            if (r, c) in dropped:
                continue
            sites[(r, c)] = q
            q += 1
    return sites


def cz_pattern(R: int, C: int, which: int, sites: dict) -> List[Tuple[int, int]]:
    """CZ pairs of pattern ``which`` (0..7) in the order H00, H11, V00, H10,
    V11, H01, V10, V01; H_ab = horizontal edges (r,c)-(r,c+1) with c%2==a and
    r%2==b, V_ab = vertical edges (r,c)-(r+1,c) with r%2==a and c%2==b."""
    order = [("H", 0, 0), ("H", 1, 1), ("V", 0, 0), ("H", 1, 0),
             ("V", 1, 1), ("H", 0, 1), ("V", 1, 0), ("V", 0, 1)]
    kind, a, b = order[which % 8]
    pairs = []
    for r in range(R):
        for c in range(C):
            if kind == "H":
                if c + 1 < C and c % 2 == a and r % 2 == b:
                    s, t = (r, c), (r, c + 1)
                else:
                    continue
            else:
                if r + 1 < R and r % 2 == a and c % 2 == b:
                    s, t = (r, c), (r + 1, c)
                else:
                    continue
            if s in sites and t in sites:
                qa, qb = sites[s], sites[t]
                pairs.append((min(qa, qb), max(qa, qb)))
    pairs.sort()
    return pairs


def grid_edges(R: int, C: int, drop: Sequence[Tuple[int, int]] = ()) -> List[Tuple[int, int]]:
    sites = grid_sites(R, C, drop)
    edges = []
    for (r, c), q in sites.items():
        if (r, c + 1) in sites:
            edges.append((q, sites[(r, c + 1)]))
        if (r + 1, c) in sites:
            edges.append((q, sites[(r + 1, c)]))
    return sorted(edges)


def supremacy_circuit(R: int, C: int, depth: int, seed: int,
                      drop: Sequence[Tuple[int, int]] = ()) -> Circuit:
    """Full depth-``depth`` circuit: cycles 0..depth-1 (cycle 0 = H layer),
    including the final CZ layer. Within a cycle the single-qubit gates come
    first (qubit ascending), then the CZs (first qubit ascending); gates in one
    cycle act on disjoint qubits."""
    sites = grid_sites(R, C, drop)
    n = len(sites)
    rng = SplitMix64(seed)
    gates: List[Gate] = [Gate("H", (q,), cycle=0) for q in range(n)]
    prev_cz = set()
    last1q = ["H"] * n
    choices = ("T", "SX", "SY")
    for t in range(1, depth):
        pairs = cz_pattern(R, C, t - 1, sites)
        cur = set()
        for a, b in pairs:
            cur.add(a)
            cur.add(b)
        for q in sorted(prev_cz - cur):
            if last1q[q] == "H":
                name = "T"
            else:
                rest = [g for g in choices if g != last1q[q]]
                name = rest[rng.next() >> 63]
            last1q[q] = name
            gates.append(Gate(name, (q,), cycle=t))
        for a, b in pairs:
            gates.append(Gate("CZ", (a, b), cycle=t))
        prev_cz = cur
    return Circuit(n, gates, dict(R=R, C=C, depth=depth, seed=seed, drop=tuple(drop)))


def drop_trailing_cz_layer(circ: Circuit) -> Circuit:
    """Remove the CZ gates of the last cycle (the paper does not simulate them,
    Sec. 3.6: they change phases, not probabilities)."""
    last = max(g.cycle for g in circ.gates)
    gates = [g for g in circ.gates if not (g.cycle == last and g.name == "CZ")]
    return Circuit(circ.n, gates, dict(circ.meta, final_cz_dropped=True))


def mirror_circuit(circ: Circuit) -> Circuit:
    """C followed by C^dagger (reverse order, each gate inverted). From |0..0>
    it returns to |0..0>. Dense gates are inverted by conjugate transpose of
    their input matrix."""
    inv = []
    for g in reversed(circ.gates):
        if g.name == "U":
            inv.append(Gate("U", g.qubits, np.ascontiguousarray(g.mat.conj().T), cycle=-2))
        else:
            inv.append(Gate(DAGGER[g.name], g.qubits, cycle=-2))
    return Circuit(circ.n, list(circ.gates) + inv, dict(circ.meta, mirrored=True))


# ---------------------------------------------------------------- other workloads
def batch_grid(n: int):
    R = int(np.floor(np.sqrt(n)))
    C = -(-n // R)
    extra = R * C - n
    drop = []
    # drop the highest-numbered sites (last row, from the right)
    for i in range(extra):
        drop.append((R - 1, C - 1 - i))
    return R, C, drop


def batch_circuit_params(index: int, n_lo: int = 14, n_hi: int = 24,
                         d_lo: int = 10, d_hi: int = 40):
    """Qubit count and depth of batch circuit ``index`` (seed 1000+index)."""
    rng = SplitMix64(1000 + index)
    n = n_lo + rng.below(n_hi - n_lo + 1)
    depth = d_lo + rng.below(d_hi - d_lo + 1)
    return n, depth, 1000 + index


def batch_circuit(index: int, **kw) -> Circuit:
    n, depth, seed = batch_circuit_params(index, **kw)
    R, C, drop = batch_grid(n)
    circ = supremacy_circuit(R, C, depth, seed, drop)
    assert circ.n == n
    circ.meta["batch_index"] = index
    return circ


def blocked_circuit(n: int, groups: Sequence[Sequence[int]], depth: int, seed: int) -> Circuit:
    """A circuit whose qubits split into independent groups: group g runs its
    own supremacy circuit on a small grid whose qubit j sits at state bit
    ``groups[g][j]``. The output is a product state over the groups, so any
    amplitude of the full state is the product of the groups' amplitudes -
    this lets an oracle check sampled amplitudes of states too large to hold."""
    all_bits = sorted(b for grp in groups for b in grp)
    assert all_bits == list(range(n)), "groups must partition the qubits"
    per_group = []
    for gi, grp in enumerate(groups):
        m = len(grp)
        R, C, drop = batch_grid(m)
        sub = supremacy_circuit(R, C, depth, seed * 1009 + gi, drop)
        per_group.append([Gate(g.name, tuple(grp[q] for q in g.qubits), g.mat, g.cycle)
                          for g in sub.gates])
    # interleave the groups cycle by cycle (they commute: disjoint qubits)
    gates = []
    for cyc in range(depth):
        for lst in per_group:
            gates.extend(g for g in lst if g.cycle == cyc)
    return Circuit(n, gates, dict(groups=[list(g) for g in groups], depth=depth, seed=seed))


def with_haar_layers(circ: Circuit, every: int, k: int, seed: int) -> Circuit:
    """Insert one Haar-random dense k-qubit gate on a uniformly drawn k-subset
    of the qubits after every ``every``-th cycle."""
    from .states import haar_unitary
    rng = SplitMix64(seed)
    last = max(g.cycle for g in circ.gates)
    out = []
    h = 0
    for cyc in range(last + 1):
        out.extend(g for g in circ.gates if g.cycle == cyc)
        if cyc > 0 and cyc % every == 0:
            pool = list(range(circ.n))
            sel = []
            for _ in range(k):  # partial Fisher-Yates
                j = rng.below(len(pool))
                sel.append(pool.pop(j))
            out.append(Gate("U", tuple(sel), haar_unitary(k, seed * 7919 + h), cycle=cyc))
            h += 1
    return Circuit(circ.n, out, dict(circ.meta, haar_every=every, haar_k=k, haar_seed=seed))


# ---------------------------------------------------------------- text format
def to_text(circ: Circuit) -> str:
    """Plain text circuit file: first line ``n <qubits>``, then one gate per
    line: ``<NAME> q0 [q1]`` for named gates, ``U k q0..q(k-1)`` followed by
    2*4^k numbers (row-major, real/imag interleaved) for dense gates."""
    lines = ["n %d" % circ.n]
    for g in circ.gates:
        if g.name == "U":
            m = np.asarray(g.mat, dtype=np.complex128)
            vals = np.empty(2 * m.size)
            vals[0::2] = m.real.ravel()
            vals[1::2] = m.imag.ravel()
            lines.append("U %d %s %s" % (g.k, " ".join(map(str, g.qubits)),
                                         " ".join("%.17g" % v for v in vals)))
        else:
            lines.append("%s %s" % (g.name, " ".join(map(str, g.qubits))))
    return "\n".join(lines) + "\n"
