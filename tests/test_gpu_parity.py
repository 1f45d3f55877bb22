"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Every case builds the same seeded input for both sides, runs the GPU
library and the oracle, and compares element by element.

Tolerances:
  * float64 states: max |d amp| <= 1e-12 for whole circuits (the target the
    project sets for the float64 path); single kernels use the bound below
    with u = 2^-53;
  * float32 states: one k-qubit cluster computes each output as a dot product
    of 2^(k+1) real terms, so |error| <= (2^(k+1) + 2) u sum_j |A_ij||b_j| <=
    (2^(k+1) + 2) u sqrt(2^k) max|amp| with u = 2^-24 (rows of the real-split
    unitary have unit norm); tests allow twice that. Whole circuits are held to
    fidelity >= 1 - 1e-6 and max |d amp| <= 4 m sqrt(2^(kmax+1)) u max|ref|
    for m passes (conftest.fp32_circuit_bound: the rounding errors of each
    pass's dot products add like a random walk, those of the passes add up).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from conftest import fp32_circuit_bound
from paper_1704_01127_amd import qsim
from supremacy_inputs import (Circuit, Gate, blocked_circuit, drop_trailing_cz_layer, haar_unitary,
                              mirror_circuit, random_state, supremacy_circuit, with_haar_layers)

pytestmark = pytest.mark.gpu

U32, U64 = 2.0 ** -24, 2.0 ** -53


def kernel_tol(dt, k, scale):
    u = U32 if dt == "c64" else U64
    return 2 * (2 ** (k + 1) + 2) * u * math.sqrt(2 ** k) * scale


def make_state(n, dt, psi=None, init="zero"):
    s = qsim.State(n, dt, init=init if psi is None else "keep")
    if psi is not None:
        s.set_amps(torch.from_numpy(psi))
    return s


def fidelity(a, b):
    a = np.asarray(a, np.complex128)
    b = np.asarray(b, np.complex128)
    return abs(np.vdot(b, a)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real)


def assert_fp32_circuit(got, ref, st, kmax):
    """A complex64 whole-circuit result against the oracle: fidelity >=
    1 - 1e-6 and max |d amp| within the float32 bound for the passes run
    (clusters of a two-cluster pass counted one by one)."""
    n_ops = max(st["n_ops"], sum(st["n_clusters_by_k"]) + st["n_diag_ops"])
    f = fidelity(got, ref)
    d = float(np.max(np.abs(np.asarray(got, np.complex128) - ref)))
    bound = fp32_circuit_bound(float(np.max(np.abs(ref))), n_ops, kmax)
    assert f >= 1 - 1e-6, f
    assert d <= bound, (d, bound, n_ops)


# ------------------------------------------------------------------ init
@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("n", [1, 5, 20])
def test_init(dt, n):
    z = make_state(n, dt).to_numpy()
    ref = np.zeros(2 ** n)
    ref[0] = 1
    assert np.array_equal(z, ref)
    u = make_state(n, dt, init="uniform").to_numpy()
    assert np.max(np.abs(u - 2.0 ** (-n / 2))) <= (1e-7 if dt == "c64" else 1e-16) * 2.0 ** (-n / 2)


# ------------------------------------------------------------------ one cluster
def target_sets(n, k, seed):
    rng = np.random.default_rng(seed)
    sets = {"low": list(range(k)), "high": list(range(n - k, n))}
    mixed = sorted(set([0, n - 1]) | set(int(q) for q in rng.choice(range(1, n - 1), k - 2, replace=False))) \
        if k >= 2 and n >= k + 1 else list(range(k))
    sets["mixed"] = mixed[:k] if len(mixed) >= k else list(range(k))
    sets["nolow"] = sorted(int(q) for q in rng.choice(range(1, n), k, replace=False)) if n > k else list(range(k))
    return sets


CLUSTER_CASES = []
for _k in range(1, 7):
    for _n in sorted({_k, _k + 1, _k + 3, 12, _k + 8}):
        if _n >= _k:
            for _pat in ("low", "high", "mixed", "nolow"):
                CLUSTER_CASES.append((_k, _n, _pat))


@pytest.fixture(params=[1, 0], ids=["staged", "direct"])
def variant(request):
    """Run with each matrix-core cluster kernel variant, then restore the default."""
    old = qsim.get_option(qsim.OPT_CLUSTER_VARIANT)
    qsim.set_option(qsim.OPT_CLUSTER_VARIANT, request.param)
    yield request.param
    qsim.set_option(qsim.OPT_CLUSTER_VARIANT, old)


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("k,n,pat", CLUSTER_CASES)
def test_apply_cluster(dt, k, n, pat, variant):
    qs = target_sets(n, k, 1000 * k + n)[pat]
    rng = np.random.default_rng(k * 7 + n)
    order = list(rng.permutation(qs))  # the ABI takes the qubits in any order
    u = haar_unitary(k, 31 * k + n)
    psi = random_state(n, 17 * n + k)
    ref = oracle.apply_dense(psi.copy(), order, u)
    s = make_state(n, dt, psi)
    s.apply_cluster(order, u)
    got = s.to_numpy()
    err = np.max(np.abs(got - ref))
    assert err <= kernel_tol(dt, k, np.max(np.abs(ref))), (err, order)


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_apply_cluster_twice_large(dt, variant):
    """Several tiles per wave and a grid that does not divide the tile count."""
    n = 21
    for k, qs in ((5, [20, 0, 7, 13, 3]), (4, [1, 2, 19, 9]), (6, [2, 3, 4, 10, 15, 20]), (3, [0, 1, 2])):
        u = haar_unitary(k, k)
        psi = random_state(n, k)
        ref = oracle.apply_dense(psi.copy(), qs, u)
        s = make_state(n, dt, psi)
        s.apply_cluster(qs, u)
        got = s.to_numpy()
        assert np.max(np.abs(got - ref)) <= kernel_tol(dt, k, np.max(np.abs(ref)))


# Two- and three-qubit clusters go through the LDS-staged vector kernel
# (64-column tiles) once n - k >= 6; targets among state bits 0..5 are the
# cases where its element-to-column mapping is least trivial.
@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("k,qs", [(2, [0, 1]), (2, [5, 9]), (2, [3, 0]), (3, [0, 1, 2]), (3, [2, 5, 6]),
                                  (3, [4, 1, 11])])
@pytest.mark.parametrize("n", [8, 9, 14])
def test_small_cluster_staged(dt, k, qs, n):
    if max(qs) >= n:
        pytest.skip("targets outside the state")
    u = haar_unitary(k, 5 * k + n)
    psi = random_state(n, 3 * n + k)
    ref = oracle.apply_dense(psi.copy(), qs, u)
    s = make_state(n, dt, psi)
    s.apply_cluster(qs, u)
    got = s.to_numpy()
    assert np.max(np.abs(got - ref)) <= kernel_tol(dt, k, np.max(np.abs(ref)))


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_small_cluster_staged_many_tiles(dt):
    """More 64-column tiles than one sweep of the grid (2^19 at n = 27, k = 2)."""
    n = 27
    for k, qs in ((2, [1, 0]), (3, [0, 2, 26])):
        u = haar_unitary(k, 77 + k)
        psi = random_state(n, 40 + k)
        ref = oracle.apply_dense(psi.copy(), qs, u)
        s = make_state(n, dt, psi)
        s.apply_cluster(qs, u)
        got = s.to_numpy()
        assert np.max(np.abs(got - ref)) <= kernel_tol(dt, k, np.max(np.abs(ref)))
        del s, got, ref, psi


# ------------------------------------------------------------------ k = 6 kernels (complex64)
@pytest.fixture(params=[0, 1, 2], ids=["realsplit", "threeprod", "fp16halves"])
def k6_kernel(request):
    old = qsim.get_option(qsim.OPT_K6_KERNEL)
    qsim.set_option(qsim.OPT_K6_KERNEL, request.param)
    yield request.param
    qsim.set_option(qsim.OPT_K6_KERNEL, old)


@pytest.mark.parametrize("n", [11, 13, 21])
@pytest.mark.parametrize("pat", ["low", "high", "mixed", "nolow"])
def test_k6_kernels(k6_kernel, n, pat):
    """Each 6-qubit float kernel at the one-cluster bound. The fp16-halves
    product drops A_lo x_lo and the split residuals (each ~2^-22 relative),
    well inside the bound's (2^(k+1) + 2) u sqrt(2^k) with u = 2^-24."""
    qs = target_sets(n, 6, 77 * n)[pat]
    u = haar_unitary(6, n + 5)
    psi = random_state(n, 3 * n)
    ref = oracle.apply_dense(psi.copy(), qs, u)
    s = make_state(n, "c64", psi)
    s.apply_cluster(qs, u)
    got = s.to_numpy()
    assert np.max(np.abs(got - ref)) <= kernel_tol("c64", 6, np.max(np.abs(ref)))


@pytest.mark.parametrize("pat", ["low", "high", "mixed", "nolow"])
def test_k6_kernel_precision_matches_fp32(pat):
    """The three 6-qubit complex64 kernels on identical inputs (a state that
    complex64 holds exactly, so the oracle's result has no input rounding):
    the fp16-halves product (operands carried to about 22 bits, three fp16
    products, fp32 accumulation) and the fp32 three-multiplication product
    stay within a factor 4 of the fp32 real-split kernel's max and RMS error.
    A factor 4 is the ratio of the halves' representation bound (2^-22
    relative) to fp32's unit roundoff (2^-24)."""
    n = 20
    errs = {}
    for trial in range(3):
        qs = target_sets(n, 6, 900 + 7 * trial)[pat]
        u = haar_unitary(6, 910 + trial)
        psi = random_state(n, 920 + trial).astype(np.complex64).astype(np.complex128)
        ref = oracle.apply_dense(psi.copy(), qs, u)
        scale = float(np.sqrt(np.mean(np.abs(ref) ** 2)))
        old = qsim.get_option(qsim.OPT_K6_KERNEL)
        try:
            for kern in (0, 1, 2):
                qsim.set_option(qsim.OPT_K6_KERNEL, kern)
                s = make_state(n, "c64", psi)
                s.apply_cluster(qs, u)
                d = np.abs(s.to_numpy().astype(np.complex128) - ref)
                e = errs.setdefault(kern, [0.0, 0.0])
                e[0] = max(e[0], float(np.max(d)) / scale)
                e[1] = max(e[1], float(np.sqrt(np.mean(d ** 2))) / scale)
                del s
        finally:
            qsim.set_option(qsim.OPT_K6_KERNEL, old)
    print("relative max / rms error by kernel (0 fp32 real-split, 1 fp32 three-product, 2 fp16 halves):",
          {k: ["%.3g" % (x / U32) + " u" for x in v] for k, v in errs.items()}, flush=True)
    for kern in (1, 2):
        assert errs[kern][0] <= 4 * errs[0][0], errs
        assert errs[kern][1] <= 4 * errs[0][1], errs
    # and all three at fp32 level: a few units of 2^-24 relative to the amplitude scale
    assert errs[0][1] <= 8 * U32


# (n, targets): the tile's top bit (bit 10 of 11) is target 5 or the highest
# column bit, with qubit 0 a target or not; the last ones are the target sets
# that are slow for the direct gather
K6_STAGED_SETS = [
    (11, [0, 1, 2, 3, 4, 5]), (11, [5, 6, 7, 8, 9, 10]), (11, [0, 2, 4, 6, 8, 10]),
    (14, [1, 2, 3, 4, 7, 13]), (14, [1, 2, 3, 4, 7, 9]), (16, [0, 1, 2, 3, 12, 15]),
    (16, [0, 1, 2, 3, 4, 6]), (21, [2, 3, 4, 10, 15, 20]), (23, [0, 1, 2, 3, 21, 22]),
    (23, [1, 2, 3, 4, 7, 14]),
]


@pytest.mark.parametrize("case", range(len(K6_STAGED_SETS)))
def test_k6_staged(case):
    """The LDS-staged fp16-halves kernel against the oracle at the one-cluster
    bound (forced variant 1), and against the direct kernel on the same input."""
    n, qs = K6_STAGED_SETS[case]
    u = haar_unitary(6, 500 + case)
    psi = random_state(n, 600 + case)
    ref = oracle.apply_dense(psi.copy(), qs, u)
    old = qsim.get_option(qsim.OPT_CLUSTER_VARIANT), qsim.get_option(qsim.OPT_K6_KERNEL)
    try:
        qsim.set_option(qsim.OPT_K6_KERNEL, 2)
        outs = {}
        for v in (1, 0):
            qsim.set_option(qsim.OPT_CLUSTER_VARIANT, v)
            s = make_state(n, "c64", psi)
            s.run_circuit([Gate("U", tuple(qs), u)], kmax=6, record_timings=True)
            recs = [r for r in s.op_timings() if r["kind"] == "cluster"]
            assert len(recs) == 1 and recs[0]["k"] == 6 and recs[0]["staged"] == (v == 1), recs
            outs[v] = s.to_numpy()
            del s
    finally:
        qsim.set_option(qsim.OPT_CLUSTER_VARIANT, old[0])
        qsim.set_option(qsim.OPT_K6_KERNEL, old[1])
    tol = kernel_tol("c64", 6, np.max(np.abs(ref)))
    assert np.max(np.abs(outs[1] - ref)) <= tol
    # same arithmetic in the same order per column: the two variants agree exactly
    assert np.array_equal(outs[1], outs[0])


@pytest.fixture(params=[0, 1], ids=["direct", "staged"])
def k6_variant(request):
    old = qsim.get_option(qsim.OPT_CLUSTER_VARIANT)
    qsim.set_option(qsim.OPT_CLUSTER_VARIANT, request.param)
    yield request.param
    qsim.set_option(qsim.OPT_CLUSTER_VARIANT, old)


@pytest.mark.parametrize("scale", [1e6, 1e-30, 0.0])
def test_k6_kernels_any_magnitude(k6_kernel, k6_variant, scale):
    """States far from unit norm, and columns that are zero: the per-column
    power-of-two scaling of the fp16 product keeps the relative error."""
    n = 14
    qs = [1, 4, 6, 9, 11, 12]  # bit 13 is not a target: each column lies in one half
    u = haar_unitary(6, 99)
    psi = random_state(n, 5)
    psi[: 2 ** (n - 1)] *= scale  # half the state rescaled (or zeroed)
    ref = oracle.apply_dense(psi.copy(), qs, u)
    s = make_state(n, "c64", psi)
    s.apply_cluster(qs, u)
    got = s.to_numpy()
    assert np.all(np.isfinite(got))
    # columns differ in scale by up to 1e30: hold each half to its own bound
    for part in (slice(0, 2 ** (n - 1)), slice(2 ** (n - 1), 2 ** n)):
        bound = kernel_tol("c64", 6, np.max(np.abs(ref[part])) if np.any(ref[part]) else 0.0)
        assert np.max(np.abs(got[part] - ref[part])) <= max(bound, 0.0), (scale, part)


def test_k6_kernels_circuit(k6_kernel, k6_variant):
    """Whole circuits with 6-qubit clusters and diagonal epilogues."""
    circ = supremacy_circuit(4, 5, 24, seed=11)
    ref = oracle.run(circ)
    s = make_state(circ.n, "c64")
    st = s.run_circuit(circ.gates, scheduler="greedy", kmax=6, fuse_diag=True)
    assert st["n_clusters_by_k"][6] > 0
    assert_fp32_circuit(s.to_numpy(), ref, st, 6)


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("kmax", [1, 3, 5, 6, 7])
def test_fold_init_matches_oracle(dt, kmax):
    """The uniform start written together with the first cluster (and its
    diagonal epilogue) in one pass gives the oracle's state, as does the
    unfolded form."""
    circ = supremacy_circuit(4, 4, 18, seed=40 + kmax)
    ref = oracle.run(circ)
    old = qsim.get_option(qsim.OPT_FOLD_INIT)
    try:
        for fold in (2, 1, 0):
            qsim.set_option(qsim.OPT_FOLD_INIT, fold)
            # the schedule depends on the folded start it is priced with
            sc = qsim.schedule(circ.n, circ.gates, qsim.C64 if dt == "c64" else qsim.C128, kmax=kmax,
                               fuse_diag=True, skip_initial_h=True)
            first_is_cluster = sc["op_kind"][0] == 0
            two = (dt == "c64" and first_is_cluster and len(sc["op_kind"]) > 1 and sc["op_kind"][1] == 0
                   and sc["op_k"][1] == 6 and sc["op_k"][0] <= 6)
            s = make_state(circ.n, dt)
            st = s.run_circuit(circ.gates, kmax=kmax, fuse_diag=True, skip_initial_h=True, record_timings=True)
            kinds = [r["kind"] for r in s.op_timings()]
            want = ("init_cluster2" if fold == 2 and two else "init_cluster" if fold and first_is_cluster else None)
            assert (want in kinds if want else not any(k.startswith("init_cluster") for k in kinds)), kinds
            got = s.to_numpy()
            if dt == "c128":
                assert np.max(np.abs(got - ref)) <= 1e-12
            else:
                assert_fp32_circuit(got, ref, st, kmax)
    finally:
        qsim.set_option(qsim.OPT_FOLD_INIT, old)


FOLD_CASES = [
    (6, (0, 1, 2, 3, 4, 5)),     # one column
    (7, (1, 2, 3, 4, 5, 6)),     # one column pair (float: columns side by side)
    (7, (0, 2, 3, 4, 5, 6)),     # qubit 0 a target (float: amplitude pairs)
    (12, (2, 5, 7, 9, 10, 11)),
    (12, (0, 5, 7, 9, 10, 11)),
    (13, (3, 8)),
    (13, (0, 12)),
    (11, (4,)),
]


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("case", range(len(FOLD_CASES)))
def test_fold_init_first_cluster(dt, case):
    """A first cluster on chosen qubits (with and without qubit 0, down to one
    column) written together with the uniform start, with diagonal gates outside
    it applied while storing."""
    n, qs = FOLD_CASES[case]
    rest = [q for q in range(n) if q not in qs]
    gates = [Gate("H", (q,)) for q in range(n)]
    gates.append(Gate("U", qs, haar_unitary(len(qs), 100 + case)))
    if len(rest) >= 2:
        gates += [Gate("CZ", (rest[0], rest[-1])), Gate("T", (rest[1],)), Gate("CZ", (qs[0], rest[0]))]
    gates += [Gate("SX", (q,)) for q in range(n)]
    circ = Circuit(n, gates)
    ref = oracle.run(circ)
    kmax = len(qs)
    sc = qsim.schedule(n, gates, kmax=kmax, fuse_diag=True, skip_initial_h=True)
    assert sc["op_kind"][0] == 0 and sorted(sc["op_qubits"][0][:sc["op_k"][0]]) == sorted(qs), sc
    old = qsim.get_option(qsim.OPT_FOLD_INIT)
    qsim.set_option(qsim.OPT_FOLD_INIT, 1)  # the first cluster alone (two: test_fold2_matches_oracle)
    try:
        s = make_state(n, dt)
        st = s.run_circuit(gates, kmax=kmax, fuse_diag=True, skip_initial_h=True, record_timings=True)
    finally:
        qsim.set_option(qsim.OPT_FOLD_INIT, old)
    kinds = [r["kind"] for r in s.op_timings() if r["kind"] != "build"]
    assert kinds[0] == "init_cluster", kinds
    got = s.to_numpy()
    if dt == "c128":
        assert np.max(np.abs(got - ref)) <= 1e-12
    else:
        assert_fp32_circuit(got, ref, st, kmax)


# (n, seed, Haar gate size): the second cluster's targets with qubit 0 or not,
# the first cluster of 6 qubits or fewer, the two overlapping or not
# (with the table form: no, 2 and 1 shared qubits in the first cases, 4 - the
# matrix-core form - in (11, 1, 2) and (11, 2, 3), target 0 in (11, 4, 6))
FOLD2_CASES = [(16, 19, 6), (11, 1, 2), (13, 7, 6), (11, 0, 6), (11, 2, 3), (11, 4, 6), (12, 21, 6), (14, 20, 6)]


@pytest.mark.parametrize("case", range(len(FOLD2_CASES)))
def test_fold2_matches_oracle(case):
    """The uniform start, a first cluster and a second 6-qubit cluster in one
    write-only pass (the second's inputs computed from the closed form, the
    first epilogue split by the second's targets) against the oracle, and
    against the same run with the three passes apart: the second cluster
    multiplied per column on the matrix cores, and (where its inputs depend on
    few column qubits) read from a table of its outputs."""
    from supremacy_inputs.circuits import batch_grid
    n, seed, hk = FOLD2_CASES[case]
    R, C, drop = batch_grid(n)
    circ = with_haar_layers(supremacy_circuit(R, C, 16, 300 + seed, drop), 4, hk, 400 + seed)
    ref = oracle.run(circ)
    opts = dict(kmax=6, fuse_diag=True, skip_initial_h=True, record_timings=True)
    old = qsim.get_option(qsim.OPT_FOLD_INIT), qsim.get_option(qsim.OPT_FOLD_TABLE)
    try:
        got, table = {}, {}
        for fold, tab in ((2, 1), (2, 0), (0, 1)):
            qsim.set_option(qsim.OPT_FOLD_INIT, fold)
            qsim.set_option(qsim.OPT_FOLD_TABLE, tab)
            s = make_state(n, "c64")
            st = s.run_circuit(circ.gates, **opts)
            recs = [r for r in s.op_timings() if r["kind"] != "build"]
            assert (recs[0]["kind"] == "init_cluster2") == (fold == 2), [r["kind"] for r in recs]
            table[(fold, tab)] = recs[0]["table"]
            got[(fold, tab)] = s.to_numpy()
    finally:
        qsim.set_option(qsim.OPT_FOLD_INIT, old[0])
        qsim.set_option(qsim.OPT_FOLD_TABLE, old[1])
    print("case", case, "table form:", table[(2, 1)])
    assert not table[(2, 0)] and not table[(0, 1)]
    bound = 2 * fp32_circuit_bound(float(np.max(np.abs(ref))), st["n_ops"] + 2, 6)
    for key in ((2, 1), (2, 0)):
        assert_fp32_circuit(got[key], ref, st, 6)
        assert np.max(np.abs(got[key] - got[(0, 1)])) <= bound


# two dense 6-qubit gates after the H layer (the whole circuit is the folded
# start): shared qubits 0, 1, 2 (the table form) and 4 (the matrix-core
# form); with a trailing CZ layer across both gates' qubits or without
FOLD2_DENSE = [((0, 2, 4, 6, 8, 10), (1, 3, 5, 7, 9, 11)),
               ((0, 1, 2, 3, 4, 5), (5, 6, 7, 8, 9, 10)),
               ((2, 4, 6, 8, 10, 12), (1, 4, 7, 10, 11, 13)),
               ((3, 4, 5, 6, 7, 8), (0, 3, 4, 5, 6, 13))]


@pytest.mark.parametrize("trailing_cz", [False, True])
@pytest.mark.parametrize("case", range(len(FOLD2_DENSE)))
def test_fold2_dense_start(case, trailing_cz):
    """The folded start of two dense 6-qubit gates without a first epilogue
    (and with or without a second one, CZ gates the schedule attaches to the
    second cluster), in the table form where the gates share at most 2 qubits
    and on the matrix cores otherwise, against the oracle."""
    n = 14
    a, b = FOLD2_DENSE[case]
    gates = [Gate("H", (q,)) for q in range(n)]
    gates.append(Gate("U", a, haar_unitary(6, 700 + case)))
    gates.append(Gate("U", b, haar_unitary(6, 710 + case)))
    if trailing_cz:
        free = [q for q in range(n) if q not in a and q not in b][0]
        only_a = [q for q in a if q not in b][0]
        only_b = [q for q in b if q not in a]
        gates += [Gate("CZ", (only_b[0], free)), Gate("CZ", (only_a, only_b[1])), Gate("CZ", (b[3], b[4]))]
        gates.append(Gate("T", (b[5],)))
        gates.append(Gate("H", (b[5],)))  # keeps the diagonal gates before it from being dropped as trailing
    circ = Circuit(n, gates)
    ref = oracle.run(circ)
    shared = len(set(a) & set(b))
    s = make_state(n, "c64")
    st = s.run_circuit(circ.gates, kmax=6, fuse_diag=True, skip_initial_h=True, record_timings=True)
    recs = [r for r in s.op_timings() if r["kind"] != "build"]
    assert recs[0]["kind"] == "init_cluster2", [r["kind"] for r in recs]
    assert recs[0]["table"] == (shared <= 2), (shared, recs[0])
    assert_fp32_circuit(s.to_numpy(), ref, st, 6)


# supremacy circuits (depth 16, seed 500 + s) whose k <= 7 schedule starts with
# two 7-qubit clusters: (n, s) sharing 2, 2 (target 0 in the second), 2, 0
# (target 0), 1 and 0 (target 0, 5 sign-flipped rows) qubits
FOLD7_CASES = [(12, 0), (12, 1), (14, 4), (16, 1), (16, 2), (18, 0)]


@pytest.mark.parametrize("case", range(len(FOLD7_CASES)))
def test_fold2_seven_qubit_start(case):
    """The uniform start and two 7-qubit clusters in one write-only pass (the
    table form: the second cluster's outputs per shared-row pattern and
    row-sign mask, combined per column) against the oracle, and against the
    same run whose start takes the first cluster only."""
    from supremacy_inputs.circuits import batch_grid
    n, seed = FOLD7_CASES[case]
    R, C, drop = batch_grid(n)
    circ = supremacy_circuit(R, C, 16, 500 + seed, drop)
    ref = oracle.run(circ)
    opts = dict(kmax=7, scheduler="learned", fuse_diag=True, skip_initial_h=True, record_timings=True)
    old = qsim.get_option(qsim.OPT_FOLD_INIT)
    try:
        got = {}
        for fold in (2, 1):
            qsim.set_option(qsim.OPT_FOLD_INIT, fold)
            s = make_state(n, "c64")
            st = s.run_circuit(circ.gates, **opts)
            recs = [r for r in s.op_timings() if r["kind"] != "build"]
            if fold == 2:
                assert recs[0]["kind"] == "init_cluster2" and recs[0]["k"] == 7 and recs[0]["table"], recs[0]
            got[fold] = s.to_numpy()
    finally:
        qsim.set_option(qsim.OPT_FOLD_INIT, old)
    assert_fp32_circuit(got[2], ref, st, 7)
    assert np.max(np.abs(got[2] - got[1])) <= 2 * fp32_circuit_bound(float(np.max(np.abs(ref))), st["n_ops"] + 2, 7)


def test_fold2_table_form_full_size():
    """The benchmarked 30-qubit grid circuit (5 x 6, depth 25, seed 0) in its
    complex64 form (learned schedule, k <= 7) starts with the table form of
    the folded start, and the whole run agrees with the same run without the
    two-cluster start (fold_table 0: the matrix-core form where the second
    cluster has 6 qubits, else the first cluster alone), element by element
    within the float32 bound."""
    circ = supremacy_circuit(5, 6, 25, 0)
    opts = dict(kmax=7, scheduler="learned", fuse_diag=True, skip_initial_h=True, skip_trailing_diag=True,
                record_timings=True)
    old = qsim.get_option(qsim.OPT_FOLD_TABLE)
    states, table = {}, {}
    try:
        for tab in (1, 0):
            qsim.set_option(qsim.OPT_FOLD_TABLE, tab)
            s = qsim.State(circ.n, "c64", kmax=7)
            st = s.run_circuit(circ.gates, **opts)
            recs = [r for r in s.op_timings() if r["kind"] != "build"]
            assert recs[0]["kind"] == ("init_cluster2" if tab else recs[0]["kind"]), [r["kind"] for r in recs]
            table[tab] = recs[0]["table"]
            states[tab] = s
    finally:
        qsim.set_option(qsim.OPT_FOLD_TABLE, old)
    assert table[1] and not table[0]
    a, b = states[1].amps, states[0].amps
    mx = float(b.abs().max())
    d = float((a - b).abs().max())
    n_ops = st["n_ops"] + 1
    print("max |d amp| %.3g, max |amp| %.3g, %d passes" % (d, mx, n_ops))
    assert d <= 2 * fp32_circuit_bound(mx, n_ops, 7), (d, mx)
    del states, a, b
    torch.cuda.empty_cache()


# ------------------------------------------------------------------ two clusters per pass (complex64)
@pytest.fixture(params=[(1, 10), (1, 11), (0, 10)], ids=["paired10", "paired11", "single"])
def pairing(request):
    """Pairing on (a tile of 10 or 11 qubits held in LDS) or off."""
    old = qsim.get_option(qsim.OPT_PAIR), qsim.get_option(qsim.OPT_PAIR_TILE)
    qsim.set_option(qsim.OPT_PAIR, request.param[0])
    qsim.set_option(qsim.OPT_PAIR_TILE, request.param[1])
    yield request.param[0]
    qsim.set_option(qsim.OPT_PAIR, old[0])
    qsim.set_option(qsim.OPT_PAIR_TILE, old[1])


PAIR_SETS = [
    ([0, 1, 2, 3, 4], [5, 6, 7, 8, 9]),        # disjoint, low
    ([0, 3, 7, 9, 12], [1, 3, 8, 12, 13]),     # overlapping, target 0 in the first
    ([9, 10, 11, 12, 13], [2, 4, 10, 12, 13]),  # high, then mixed
    ([1, 2, 6], [0, 5, 7, 8]),                  # padded (3 and 4 qubits), target 0 in the second
    ([4, 5, 6, 7, 8], [4, 5, 6, 7, 8]),        # the same qubits twice
    ([1, 2, 3, 4, 5], [6, 7, 8, 9, 10]),       # ten targets above bit 0 (the 11-qubit tile)
]


@pytest.mark.parametrize("n", [11, 14, 21])
@pytest.mark.parametrize("case", range(len(PAIR_SETS)))
def test_pair_of_dense_clusters(pairing, n, case):
    """Two dense clusters in a row: one pass (pairing) or two; the bound is
    twice the one-cluster bound (two products, each ~2^-22 relative)."""
    qa, qb = PAIR_SETS[case]
    qa = [q for q in qa if q < n]
    qb = [q for q in qb if q < n]
    ua, ub = haar_unitary(len(qa), 7 * n + case), haar_unitary(len(qb), 11 * n + case)
    psi = random_state(n, 13 * n + case)
    ref = oracle.apply_dense(oracle.apply_dense(psi.copy(), qa, ua), qb, ub)
    gates = [("U", tuple(qa), ua), ("U", tuple(qb), ub)]
    two_ops = len(qsim.schedule(n, gates, kmax=5)["op_kind"]) == 2  # else one cluster holds both
    s = make_state(n, "c64", psi)
    s.run_circuit(gates, kmax=5, record_timings=True)
    kinds = [r["kind"] for r in s.op_timings()]
    assert ("pair" in kinds) == (bool(pairing) and two_ops), kinds
    got = s.to_numpy()
    assert np.max(np.abs(got - ref)) <= 2 * kernel_tol("c64", 5, np.max(np.abs(ref)))


@pytest.mark.parametrize("kmax", [3, 4, 5])
@pytest.mark.parametrize("fuse", [False, True])
def test_pair_circuits_match_oracle(pairing, kmax, fuse):
    """Whole circuits with clusters paired (diagonal epilogues on both)."""
    circ = with_haar_layers(supremacy_circuit(4, 4, 22, seed=60 + kmax), 7, 3, 5)
    ref = oracle.run(circ)
    s = make_state(circ.n, "c64")
    st = s.run_circuit(circ.gates, kmax=kmax, fuse_diag=fuse, skip_initial_h=True)
    assert_fp32_circuit(s.to_numpy(), ref, st, kmax)


# ------------------------------------------------------------------ diagonal layer
@pytest.mark.parametrize("dt", ["c64", "c128"])
# 8: fewer windows than one wave's step; 25: more windows than one sweep of the grid
@pytest.mark.parametrize("n", [1, 2, 3, 8, 9, 16, 25])
def test_apply_diag(dt, n):
    rng = np.random.default_rng(n)
    pairs = []
    if n >= 2:
        perm = list(rng.permutation(n))
        pairs = [(int(perm[2 * i]), int(perm[2 * i + 1])) for i in range(n // 2)]
        pairs.append((0, n - 1))
        if n >= 3:
            pairs.append((1, 2))
    phases = [(int(q), float(rng.uniform(-np.pi, np.pi))) for q in rng.choice(n, min(n, 5), replace=False)]
    phases.append((0, np.pi / 4))
    psi = random_state(n, n + 5)
    ref = psi.copy()
    for a, b in pairs:
        oracle.apply_named(ref, "CZ", a, b)
    for q, th in phases:
        oracle.apply_dense(ref, (q,), np.diag([1.0, np.exp(1j * th)]))
    s = make_state(n, dt, psi)
    s.apply_diag(pairs, phases)
    got = s.to_numpy()
    assert np.max(np.abs(got - ref)) <= (8 * U32 if dt == "c64" else 8 * U64) * np.max(np.abs(ref))


# ------------------------------------------------------------------ per-gate kernels
NAMED = ["H", "T", "SX", "SY", "X", "Y", "Z", "TDG", "SXDG", "SYDG"]


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("name", NAMED + ["CZ", "U"])
def test_apply_gate(dt, name):
    n = 11
    psi = random_state(n, 3)
    ref = psi.copy()
    s = make_state(n, dt, psi)
    if name == "CZ":
        targets = [(0, 1), (n - 1, 0), (4, 9), (n - 2, n - 1)]
    elif name == "U":
        targets = [(3, 0), (n - 1, 5, 2)]
    else:
        targets = [(0,), (5,), (n - 1,)]
    for t in targets:
        if name == "U":
            u = haar_unitary(len(t), len(t))
            s.apply_gate(("U", t, u))
            oracle.apply_dense(ref, t, u)
        else:
            s.apply_gate((name, t))
            oracle.apply_named(ref, name, t[0], t[1] if len(t) > 1 else -1)
    got = s.to_numpy()
    assert np.max(np.abs(got - ref)) <= kernel_tol(dt, 3, 1.0) * len(targets)


def test_phase_gate():
    n = 6
    psi = random_state(n, 4)
    s = make_state(n, "c128", psi)
    s.apply_gate(("PHASE", (2,), 0.3))
    ref = oracle.apply_dense(psi.copy(), (2,), np.diag([1, np.exp(0.3j)]))
    assert np.max(np.abs(s.to_numpy() - ref)) <= 1e-15


# ------------------------------------------------------------------ 7-qubit clusters
def seven_qubit_gates(qs, others, seed, epilogue=True):
    """Gates on the seven qubits qs only (random named single-qubit gates, CZ
    layers on random pairings, a Haar 4-qubit gate, a closing H layer), which
    a kmax = 7 schedule fuses into one cluster; then diagonal gates on other
    qubits and between qs and others (its epilogue with fuse_diag)."""
    rng = np.random.default_rng(seed)
    gates = []
    for layer in range(5):
        for q in qs:
            gates.append(Gate(str(rng.choice(["H", "SX", "SY", "T", "X", "Y", "Z", "TDG"])), (q,)))
        perm = [int(x) for x in rng.permutation(qs)]
        gates.extend(Gate("CZ", (a, b)) for a, b in zip(perm[0::2], perm[1::2]))
    sub = tuple(int(x) for x in rng.choice(qs, 4, replace=False))
    gates.append(Gate("U", sub, haar_unitary(4, seed)))
    gates.extend(Gate("H", (q,)) for q in qs)
    if epilogue and len(others) >= 3:
        gates += [Gate("CZ", (qs[1], others[0])), Gate("T", (others[1],)), Gate("CZ", (others[1], others[2])),
                  Gate("Z", (others[2],)),
                  Gate("CZ", (others[0], qs[5])), Gate("TDG", (others[0],))]
    return gates


SEVEN_SETS = {
    "middle": lambda n: list(range(n // 2 - 3, n // 2 + 4)),
    "low": lambda n: list(range(7)),                        # qubit 0 a target (16-byte accesses), columns spread
    "high": lambda n: list(range(n - 7, n)),
    "spread": lambda n: sorted({0, 2, n // 3, n // 2, n // 2 + 1, n - 2, n - 1}),
    "nolow": lambda n: sorted({1, 3, 4, n // 2, n - 4, n - 3, n - 1}),
}


@pytest.mark.parametrize("n", [12, 13, 17, 21])
@pytest.mark.parametrize("pat", sorted(SEVEN_SETS))
@pytest.mark.parametrize("fuse", [False, True])
def test_seven_qubit_cluster(n, pat, fuse):
    """One 7-qubit cluster (fp16 halves of Re M and Im M on the matrix cores)
    on a random state, with and without a diagonal epilogue, against the
    oracle's gate-by-gate result at the one-cluster bound for k = 7. n = 12
    is the smallest state (one wave tile of 32 columns); 21 gives every wave
    several tiles."""
    qs = SEVEN_SETS[pat](n)
    others = [q for q in range(n) if q not in qs]
    gates = seven_qubit_gates(qs, others, 100 * n + len(pat), epilogue=True)
    psi = random_state(n, 13 * n + len(pat))
    ref = oracle.apply(psi.copy(), Circuit(n, gates))
    s = make_state(n, "c64", psi)
    st = s.run_circuit(gates, scheduler="greedy", kmax=7, fuse_diag=fuse, record_timings=True)
    assert st["n_clusters_by_k"][7] == 1 and sum(st["n_clusters_by_k"]) == 1, st
    assert st["n_ops"] == (1 if fuse else 2), st
    ops = [r for r in s.op_timings() if r["kind"] == "cluster"]
    assert ops[0]["k"] == 7 and ops[0]["qubits"] == qs and ops[0]["epi"] == fuse, ops
    got = s.to_numpy()
    err = np.max(np.abs(got - ref))
    # the epilogue pass (without fuse) is exact up to fp32 products
    bound = kernel_tol("c64", 7, np.max(np.abs(ref))) + (0 if fuse else 4 * U32 * np.max(np.abs(ref)))
    assert err <= bound, (err, bound, qs)


@pytest.mark.parametrize("pat", sorted(SEVEN_SETS))
def test_seven_qubit_cluster_precision(pat):
    """The 7-qubit kernel's error on a state complex64 holds exactly (no input
    rounding): max and RMS error against the oracle stay within a factor 2 of
    the 6-qubit fp16-halves kernel's on the same kind of input, scaled by the
    square root of the dot-product length (sqrt 2); both far below plain fp16
    arithmetic (2^-11 relative)."""
    n = 16
    qs = SEVEN_SETS[pat](n)
    gates = seven_qubit_gates(qs, [], 7 + len(pat), epilogue=False)
    psi = random_state(n, 5 + len(pat)).astype(np.complex64).astype(np.complex128)
    ref = oracle.apply(psi.copy(), Circuit(n, gates))
    s = make_state(n, "c64", psi)
    st = s.run_circuit(gates, scheduler="greedy", kmax=7)
    assert st["n_clusters_by_k"][7] == 1
    d7 = np.abs(s.to_numpy() - ref)
    # the same gates without the last qubit's share: a 6-qubit cluster
    q6 = qs[:6]
    g6 = [g for g in gates if set(g.qubits) <= set(q6)]
    ref6 = oracle.apply(psi.copy(), Circuit(n, g6))
    s6 = make_state(n, "c64", psi)
    st6 = s6.run_circuit(g6, scheduler="greedy", kmax=6)
    assert st6["n_clusters_by_k"][6] == 1
    d6 = np.abs(s6.to_numpy() - ref6)
    mx = float(np.max(np.abs(ref)))
    assert d7.max() <= 2 * np.sqrt(2) * max(d6.max(), 2 * U32 * mx), (d7.max(), d6.max())
    rms7, rms6 = np.sqrt(np.mean(d7 ** 2)), np.sqrt(np.mean(d6 ** 2))
    assert rms7 <= 2 * np.sqrt(2) * rms6, (rms7, rms6)
    assert d7.max() <= 2.0 ** -16 * mx


def test_seven_qubit_fused_stats():
    """The 7-qubit kernel's STATS form: a run whose last op is a 7-qubit
    cluster returns the same norm, sum p^2 and entropy from the kernel's own
    sums as the separate reduction."""
    n = 18
    qs = SEVEN_SETS["middle"](n)
    gates = seven_qubit_gates(qs, [0, 1, 2], 3, epilogue=True)
    psi = random_state(n, 3)
    ref = make_state(n, "c64", psi)
    ref.run_circuit(gates, kmax=7, fuse_diag=True)
    want = ref.probs()
    s = make_state(n, "c64", psi)
    s.run_circuit(gates, kmax=7, fuse_diag=True, fused_stats=True)
    s.amps.zero_()
    torch.cuda.synchronize()
    got = s.probs()
    for a, b in zip(got, want):
        assert abs(a - b) <= 1e-12 * max(1.0, abs(b)), (got, want)
    onorm, osp2, oent = oracle.stats(oracle.apply(psi.copy(), Circuit(n, gates)))
    assert abs(got[0] - onorm) <= 1e-5 and abs(got[2] - oent) <= 1e-4


def test_seven_qubit_circuits():
    """Whole circuits with kmax = 7 against the oracle: a 20-qubit depth-25
    grid circuit (greedy and learned schedules, diagonal epilogues, the
    uniform start folded into a first 7-qubit cluster) and one with Haar
    5-qubit gates; the same runs on a complex128 state are capped at 6 qubits."""
    for circ in (supremacy_circuit(4, 5, 25, 3), with_haar_layers(supremacy_circuit(4, 5, 24, 4), 6, 5, 9)):
        ref = oracle.run(circ)
        for sched in ("greedy", "learned"):
            s = make_state(circ.n, "c64")
            st = s.run_circuit(circ.gates, scheduler=sched, kmax=7, fuse_diag=True, skip_initial_h=True)
            assert_fp32_circuit(s.to_numpy(), ref, st, 7)
            if sched == "greedy":
                assert st["n_clusters_by_k"][7] > 0, st
        s = make_state(circ.n, "c128")
        st = s.run_circuit(circ.gates, scheduler="greedy", kmax=7, fuse_diag=True, skip_initial_h=True)
        assert st["n_clusters_by_k"][7] == 0 and st["n_clusters_by_k"][6] > 0, st
        assert np.max(np.abs(s.to_numpy() - ref)) <= 1e-12


# ------------------------------------------------------------------ whole circuits
RUN_CASES = [
    dict(scheduler="per_gate"),
    dict(scheduler="greedy", kmax=1),
    dict(scheduler="greedy", kmax=2),
    dict(scheduler="greedy", kmax=3),
    dict(scheduler="greedy", kmax=4),
    dict(scheduler="greedy", kmax=5),
    dict(scheduler="greedy", kmax=6),
    dict(scheduler="greedy", kmax=3, fuse_diag=True),
    dict(scheduler="greedy", kmax=4, fuse_diag=True),
    dict(scheduler="greedy", kmax=5, fuse_diag=True),
    dict(scheduler="greedy", kmax=6, fuse_diag=True),
    dict(scheduler="greedy", kmax=5, fuse_diag=True, skip_initial_h=True),
    dict(scheduler="greedy", kmax=7),                    # complex128: capped at 6
    dict(scheduler="greedy", kmax=7, fuse_diag=True, skip_initial_h=True),
]


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("case", range(len(RUN_CASES)))
def test_run_circuit_16q(dt, case, variant):
    opts = RUN_CASES[case]
    circ = supremacy_circuit(4, 4, 20, seed=case)
    ref = oracle.run(circ)
    s = make_state(circ.n, dt)
    st = s.run_circuit(circ.gates, **opts)
    got = s.to_numpy()
    if dt == "c128":
        assert np.max(np.abs(got - ref)) <= 1e-12
    else:
        assert_fp32_circuit(got, ref, st, opts.get("kmax", 1))
    assert st["n_gates_applied"] <= len(circ.gates)


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_skip_trailing_diag_keeps_probabilities(dt):
    circ = supremacy_circuit(4, 4, 18, seed=5)
    ref = oracle.run(circ)
    s = make_state(circ.n, dt)
    st = s.run_circuit(circ.gates, kmax=4, fuse_diag=True, skip_trailing_diag=True)
    got = s.to_numpy()
    assert st["n_gates_applied"] < len(circ.gates)
    tol = 1e-14 if dt == "c128" else 1e-6
    assert np.max(np.abs(np.abs(got) ** 2 - np.abs(ref) ** 2)) <= tol * np.max(np.abs(ref) ** 2) * 10


def test_dense_gates_in_circuit():
    from supremacy_inputs import with_haar_layers
    circ = with_haar_layers(supremacy_circuit(3, 4, 20, 0), 8, 5, 3)
    ref = oracle.run(circ)
    for dt in ("c64", "c128"):
        for opts in (dict(scheduler="per_gate"), dict(kmax=3), dict(kmax=6, fuse_diag=True)):
            s = make_state(circ.n, dt)
            st = s.run_circuit(circ.gates, **opts)
            got = s.to_numpy()
            if dt == "c128":
                assert np.max(np.abs(got - ref)) <= 1e-12
            else:
                assert_fp32_circuit(got, ref, st, 6)  # the Haar gates are 5-qubit clusters even per gate


@pytest.mark.parametrize("seed", range(10))
def test_20q_depth25_per_gate_float64(seed):
    """4x5 grid, depth 25, complex128, one gate at a time: max |d amp| <= 1e-12."""
    circ = supremacy_circuit(4, 5, 25, seed)
    ref = oracle.run(circ)
    s = make_state(20, "c128")
    s.run_circuit(circ.gates, scheduler="per_gate")
    got = s.to_numpy()
    assert np.max(np.abs(got - ref)) <= 1e-12
    # the same through the fused float64 and float32 forms
    s2 = make_state(20, "c128")
    s2.run_circuit(circ.gates, kmax=5, fuse_diag=True)
    assert np.max(np.abs(s2.to_numpy() - ref)) <= 1e-12
    for kmax in (5, 6, 7):
        s3 = make_state(20, "c64")
        st = s3.run_circuit(circ.gates, kmax=kmax, scheduler="learned", fuse_diag=True, skip_initial_h=True)
        assert_fp32_circuit(s3.to_numpy(), ref, st, kmax)


# ------------------------------------------------------------------ bit permutation
PERM_CASES = [
    (5, [0, 4], [4, 0]), (11, [0, 1, 2], [2, 0, 1]), (12, list(range(12)), list(range(11, -1, -1))),
    (13, [3, 5, 7, 9, 11, 0], [0, 11, 9, 7, 5, 3]), (21, [20, 0], [0, 20]),
    (21, [2, 4, 6, 15, 17, 20], [15, 17, 20, 2, 4, 6]),
    (22, [0, 1, 2, 3, 4, 5, 16, 17, 18, 19, 20, 21], [16, 17, 18, 19, 20, 21, 0, 1, 2, 3, 4, 5]),
    (23, [9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 22], [22, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19]),
]


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("case", range(len(PERM_CASES)))
def test_permute_qubits(dt, case):
    """Bit relabelling (data movement only): bit-exact against the oracle's
    permutation of the same stored amplitudes; tiles of the moving bits plus
    the lowest fixed ones, any number of tiles."""
    n, src, dst = PERM_CASES[case]
    psi = random_state(n, 70 + case)
    s = make_state(n, dt, psi)
    held = s.to_numpy().astype(np.complex128)
    s.permute_qubits(src, dst)
    got = s.to_numpy().astype(np.complex128)
    np.testing.assert_array_equal(got, oracle.permute_bits(held, src, dst))
    s.permute_qubits(dst, src)
    np.testing.assert_array_equal(s.to_numpy().astype(np.complex128), held)


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("kmax", [4, 6, 7])
def test_map_qubits_matches_oracle(dt, kmax):
    """QSIM_OPT_MAP_QUBITS: the run applies relabelled gates from the uniform
    state and one permutation pass restores the order; the state (and the
    fused sums) equal the oracle's."""
    circ = with_haar_layers(supremacy_circuit(4, 5, 25, seed=3), 8, 5, 9)
    ref = oracle.run(circ)
    old = qsim.get_option(qsim.OPT_MAP_QUBITS)
    qsim.set_option(qsim.OPT_MAP_QUBITS, 1)
    try:
        s = make_state(20, dt)
        st = s.run_circuit(circ.gates, kmax=kmax, fuse_diag=True, skip_initial_h=True, record_timings=True,
                           fused_stats=True)
        kinds = [r["kind"] for r in s.op_timings()]
        norm, s2, ent = s.probs()
    finally:
        qsim.set_option(qsim.OPT_MAP_QUBITS, old)
    assert kinds[-1] == "permute", kinds  # this circuit's layout moves qubits
    got = s.to_numpy()
    if dt == "c128":
        assert np.max(np.abs(got - ref)) <= 1e-12
    else:
        assert_fp32_circuit(got, ref, st, kmax)
    on, os2, oent = oracle.stats(ref)
    tol = 1e-12 if dt == "c128" else 1e-5
    assert abs(norm - on) <= tol and abs(s2 - os2) <= tol * os2 * 10 and abs(ent - oent) <= tol * 20


def test_permute_qubits_errors():
    s = make_state(8, "c64")
    for src, dst in (([0, 1], [1, 2]), ([0, 0], [1, 1]), ([8], [8]), (list(range(13)), list(range(13)))):
        with pytest.raises(qsim.QsimError):
            s.permute_qubits(src, dst)


# ------------------------------------------------------------------ reductions
@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_probs_and_compare(dt):
    circ = supremacy_circuit(4, 5, 25, 7)
    ref = oracle.run(circ)
    norm_o, s2_o, ent_o = oracle.stats(ref)
    s = make_state(20, dt)
    s.run_circuit(circ.gates, kmax=5, fuse_diag=True)
    out = torch.empty(2 ** 20, dtype=torch.float64 if dt == "c128" else torch.float32, device="cuda")
    norm, s2, ent = s.probs(out)
    tol = 1e-12 if dt == "c128" else 1e-5
    assert abs(norm - norm_o) <= tol and abs(ent - ent_o) <= tol * 20 and abs(s2 - s2_o) <= tol * s2_o
    # the reduction alone: against the exact statistics of the state's own amplitudes
    # (float states take ln of the mantissa in float: <= ~1.4e-7 absolute per unit of
    # probability)
    pg = np.abs(s.to_numpy().astype(np.complex128)) ** 2
    ent_g = float(-np.sum(pg[pg > 0] * np.log(pg[pg > 0])))
    assert abs(ent - ent_g) <= (1e-12 if dt == "c128" else 3e-7)
    assert abs(norm - float(np.sum(pg))) <= (1e-12 if dt == "c128" else 1e-9)
    p = out.cpu().numpy()
    assert np.max(np.abs(p - np.abs(ref) ** 2)) <= (1e-15 if dt == "c128" else 1e-6 * np.max(np.abs(ref) ** 2))
    refd = torch.from_numpy(ref).cuda()
    f, md = s.compare(refd)
    got = s.to_numpy()
    assert abs(f - fidelity(got, ref)) <= 1e-12
    assert abs(md - np.max(np.abs(got - ref))) <= 1e-12
    if dt == "c128":
        assert md <= 1e-12 and abs(f - 1) <= 1e-12


# ------------------------------------------------------------------ larger states
def test_22q_full_circuit_float32():
    """4x6 grid minus two sites (22 qubits), depth 25, float32 fused vs oracle."""
    circ = supremacy_circuit(4, 6, 25, 11, drop=[(3, 5), (3, 4)])
    assert circ.n == 22
    ref = oracle.run(circ)
    for opts in (dict(kmax=5, fuse_diag=True), dict(kmax=4), dict(kmax=6, fuse_diag=True), dict(kmax=7, fuse_diag=True)):
        s = make_state(22, "c64")
        st = s.run_circuit(circ.gates, **opts)
        assert_fp32_circuit(s.to_numpy(), ref, st, opts["kmax"])


def _blocked_30q():
    groups = [[0, 5, 10, 15, 20, 25], [1, 6, 11, 16, 21, 26], [2, 7, 12, 17, 22, 27],
              [3, 8, 13, 18, 23, 28], [4, 9, 14, 19, 24, 29]]
    return blocked_circuit(30, groups, 20, seed=3), groups


def _product_amplitudes(circ, groups, idx):
    amps = np.ones(len(idx), np.complex128)
    for gi, grp in enumerate(groups):
        sub = Circuit(len(grp), [Gate(g.name, tuple(grp.index(q) for q in g.qubits), g.mat)
                                 for g in circ.gates if set(g.qubits) <= set(grp)])
        psi = oracle.run(sub)
        loc = np.zeros(len(idx), np.int64)
        for j, q in enumerate(grp):
            loc |= ((idx >> q) & 1) << j
        amps *= psi[loc]
    return amps


@pytest.mark.parametrize("dt,opts", [("c64", dict(kmax=5, fuse_diag=True)), ("c64", dict(kmax=6)),
                                     ("c64", dict(kmax=7, scheduler="learned", fuse_diag=True, skip_initial_h=True)),
                                     ("c128", dict(kmax=5, fuse_diag=True)), ("c128", dict(scheduler="per_gate"))])
def test_30q_product_state_sampled(dt, opts):
    """30 qubits in five independent 6-qubit groups interleaved across all
    bit positions: every amplitude is a product of group amplitudes, which
    the oracle computes exactly; 65536 sampled indices are compared."""
    circ, groups = _blocked_30q()
    s = make_state(30, dt)
    s.run_circuit(circ.gates, **opts)
    s.sync()
    rng = np.random.default_rng(0)
    idx = np.concatenate([rng.integers(0, 2 ** 30, 65536 - 2), [0, 2 ** 30 - 1]]).astype(np.int64)
    ref = _product_amplitudes(circ, groups, idx)
    got = s.amps[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.complex128)
    scale = np.max(np.abs(ref))
    err = np.max(np.abs(got - ref))
    assert err <= (1e-12 if dt == "c128" else 2e-5 * scale), err
    norm, _, _ = s.probs()
    assert abs(norm - 1) <= (1e-12 if dt == "c128" else 1e-5)
    del s
    torch.cuda.empty_cache()


@pytest.mark.parametrize("opts", [dict(kmax=7, scheduler="learned", fuse_diag=True, skip_initial_h=True),
                                  dict(kmax=6, scheduler="learned", fuse_diag=True, skip_initial_h=True),
                                  dict(kmax=5, fuse_diag=True)])
def test_34q_product_state_sampled(opts):
    """34 qubits (the largest complex64 state: 128 GiB) in six independent
    groups interleaved across all bit positions (qubit q in group q mod 6),
    run in the benchmark's form and at k <= 5; 65536 sampled amplitudes
    against the oracle's exact products."""
    groups = [[q for q in range(34) if q % 6 == r] for r in range(6)]
    circ = blocked_circuit(34, groups, 18, seed=5)
    s = make_state(34, "c64")
    s.run_circuit(circ.gates, **opts)
    s.sync()
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.integers(0, 2 ** 34, 65536 - 2), [0, 2 ** 34 - 1]]).astype(np.int64)
    ref = _product_amplitudes(circ, groups, idx)
    got = s.amps[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.complex128)
    err = np.max(np.abs(got - ref))
    assert err <= 2e-5 * np.max(np.abs(ref)), err
    norm, _, _ = s.probs()
    assert abs(norm - 1) <= 1e-5
    del s
    torch.cuda.empty_cache()


def test_30q_depth25_mirror_float32():
    """5x6 grid, depth 25, followed by its inverse: the float32 fused run must
    return to |0...0> (the workload the benchmark times)."""
    circ = supremacy_circuit(5, 6, 25, 0)
    s = make_state(30, "c64")
    s.run_circuit(mirror_circuit(circ).gates, kmax=5, fuse_diag=True)
    a0 = s.amps[0].item()
    assert abs(a0) ** 2 >= 1 - 1e-6
    norm, _, _ = s.probs()
    assert abs(norm - 1) <= 1e-5
    del s
    torch.cuda.empty_cache()


# ------------------------------------------------------------------ reductions fused into the last pass
FUSED_CASES = [
    (6, [10, 11, 12, 13, 14, 15], 0), (6, [0, 3, 7, 9, 12, 14], 0),  # direct k = 6, without / with qubit 0
    (5, [9, 10, 11, 12, 13], 0), (5, [0, 4, 8, 12, 14], 0),          # direct k = 5
    (4, [3, 8, 11, 15], 0), (4, [0, 5, 9, 13], 0),                   # direct k = 4 (forced)
    (4, [3, 8, 11, 15], 1),                                          # staged: not fused, recomputed
    (3, [3, 8, 11], 0), (3, [0, 5, 9], 0), (2, [4, 10], 0),          # staged vector-ALU kernel, k = 2, 3
]


@pytest.mark.parametrize("n", [12, 16, 22])
@pytest.mark.parametrize("k,qs,variant", FUSED_CASES)
def test_fused_stats(n, k, qs, variant):
    """A run whose last op is a cluster applied by a direct matrix-core kernel
    (k = 4..6) or the staged vector-ALU kernel (k = 2, 3)
    with fused_stats: the norm, sum p^2 and entropy of the stored state come
    from that kernel and equal the separate reduction's. The probe: the state
    is then overwritten directly; the fused path still reports the run's sums
    (they describe the state the run left), the staged kernel's run reads the
    overwritten state. At n = 12 some waves of the launch own no tile."""
    if max(qs) >= n:
        pytest.skip("targets outside the state")
    old = qsim.get_option(qsim.OPT_CLUSTER_VARIANT)
    qsim.set_option(qsim.OPT_CLUSTER_VARIANT, variant)
    try:
        u = haar_unitary(k, 3 * k + n)
        psi = random_state(n, 7 * n + k)
        gates = [("CZ", (1, 2)), ("U", tuple(qs), u)]
        ref = make_state(n, "c64", psi)
        ref.run_circuit(gates, kmax=k, fuse_diag=True)
        want = ref.probs()
        s = make_state(n, "c64", psi)
        s.run_circuit(gates, kmax=k, fuse_diag=True, fused_stats=True)
        s.amps.zero_()
        torch.cuda.synchronize()
        got = s.probs()
        if variant == 0:
            for a, b in zip(got, want):
                assert abs(a - b) <= 1e-12 * max(1.0, abs(b)), (got, want)
            assert abs(got[0] - 1) <= 1e-5
            # a call that rewrites the partial sums ends the fused result
            s.probs(torch.empty(2 ** n, dtype=torch.float32, device="cuda"))
            assert s.probs()[0] == 0.0
        else:
            assert got == (0.0, 0.0, 0.0)
    finally:
        qsim.set_option(qsim.OPT_CLUSTER_VARIANT, old)


def test_fused_stats_cleared_by_state_changes():
    """After a fused run, any call that changes the state recomputes."""
    n = 14
    u = haar_unitary(6, 1)
    s = make_state(n, "c64", random_state(n, 2))
    s.run_circuit([("U", (8, 9, 10, 11, 12, 13), u)], kmax=6, fused_stats=True)
    s.apply_cluster([0], np.array([[0, 1], [1, 0]], np.complex128))
    s.amps.zero_()
    torch.cuda.synchronize()
    assert s.probs()[0] == 0.0
    # a copy into the state through the binding (set_amps) drops the sums too
    s.run_circuit([("U", (8, 9, 10, 11, 12, 13), u)], kmax=6, fused_stats=True)
    s.set_amps(torch.zeros(2 ** n, dtype=torch.complex64))
    assert s.probs() == (0.0, 0.0, 0.0)


BENCH_FORM = dict(scheduler="learned", fuse_diag=True, skip_initial_h=True)


@pytest.mark.parametrize("R,C,drop,dt,kmax,bar", [
    (5, 6, (), "c64", 7, 1e-6),
    (5, 6, (), "c64", 6, 1e-6),
    (5, 6, (), "c128", 5, 1e-12),
    (5, 7, ((4, 6),), "c64", 7, 1e-6),
], ids=["30q-f32", "30q-f32-k6", "30q-f64", "34q-f32"])
def test_mirror_bench_form(R, C, drop, dt, kmax, bar):
    """The depth-25 grid circuits followed by their inverse, run the way the
    benchmark runs them (learned schedule, diagonal epilogues, the leading H
    layer as the uniform start folded into the first clusters): the state
    must return to |0...0> (float32 >= 1 - 1e-6, float64 >= 1 - 1e-12) with
    unit norm; at 34 qubits no host oracle fits, this is its whole-circuit pin."""
    circ = mirror_circuit(supremacy_circuit(R, C, 25, 0, list(drop)))
    s = make_state(circ.n, dt)
    st = s.run_circuit(circ.gates, kmax=kmax, **BENCH_FORM)
    assert st["n_ops"] > 0
    a0 = s.amps[0].item()
    assert abs(a0) ** 2 >= 1 - bar, abs(a0) ** 2
    norm, _, _ = s.probs()
    assert abs(norm - 1) <= (1e-12 if dt == "c128" else 1e-5)
    del s
    torch.cuda.empty_cache()


# ------------------------------------------------------------------ errors
def test_argument_errors():
    s = make_state(6, "c64")
    with pytest.raises(qsim.QsimError, match="INVALID"):
        s.apply_cluster([0, 6], np.eye(4))
    with pytest.raises(qsim.QsimError, match="INVALID"):
        s.apply_cluster([1, 1], np.eye(4))
    with pytest.raises(qsim.QsimError, match="UNSUPPORTED"):
        s.run_circuit([("H", (0,))], kmax=8)
    with pytest.raises(qsim.QsimError, match="INVALID"):
        s.apply_diag([(2, 2)])
    s.sync()
