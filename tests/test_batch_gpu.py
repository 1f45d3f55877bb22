"""Parity of the batched persistent launch (through the C ABI) with the CPU
oracle: many circuits of uneven sizes in one launch, each compared with the
oracle's float64 state (complex64 whole-circuit bar: fidelity >= 1 - 1e-6,
max |d amp| within the float32 bound of conftest.fp32_circuit_bound for the
circuit's passes), plus the launch's own controls (grid, padding, repeat
runs) and its bounded dependency wait."""
import numpy as np
import pytest

import oracle
from conftest import fp32_circuit_bound
from paper_1704_01127_amd import qsim
from supremacy_inputs import batch_circuit, haar_unitary, supremacy_circuit, with_haar_layers
from supremacy_inputs.circuits import batch_grid

pytestmark = pytest.mark.gpu


def fidelity(a, b):
    a = np.asarray(a, np.complex128)
    b = np.asarray(b, np.complex128)
    return abs(np.vdot(b, a)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real)


def small_batch(count, n_lo=11, n_hi=16, seed0=0):
    """Seeded supremacy circuits with n in [n_lo, n_hi], depth in [10, 40]."""
    circs = []
    for i in range(count):
        circs.append(batch_circuit(seed0 + i, n_lo=n_lo, n_hi=n_hi))
    return circs


def passes(batch, c):
    """Passes over the state a batched circuit takes: its ops as the batch
    schedules them, plus the initialisation."""
    sc = qsim.schedule(c.n, c.gates, kmax=batch.kmax, scheduler="greedy", fuse_diag=True, skip_initial_h=True)
    return len(sc["op_kind"]) + 1


def check_against_oracle(batch, circs, skip_trailing_diag=False, index=None):
    for j, c in enumerate(circs):
        i = j if index is None else index[j]
        ref = oracle.run(c)
        got = batch.states[i].cpu().numpy().astype(np.complex128)
        if skip_trailing_diag:  # probabilities only are defined then
            p, pr = np.abs(got) ** 2, np.abs(ref) ** 2
            assert np.max(np.abs(p - pr)) <= 1e-6 * np.max(pr) * 10, i
            continue
        f = fidelity(got, ref)
        d = np.max(np.abs(got - ref))
        bound = fp32_circuit_bound(float(np.max(np.abs(ref))), passes(batch, c), 6)
        assert f >= 1 - 1e-6 and d <= bound, (i, c.n, f, d, bound)


@pytest.fixture(autouse=True)
def _reset_options():
    fold = qsim.get_option(qsim.OPT_FOLD_INIT)
    order = qsim.get_option(qsim.OPT_BATCH_ORDER)
    yield
    qsim.set_option(qsim.OPT_BATCH_GRID, 0)
    qsim.set_option(qsim.OPT_BATCH_PAD, 0)
    qsim.set_option(qsim.OPT_FOLD_INIT, fold)
    qsim.set_option(qsim.OPT_BATCH_ORDER, order)


@pytest.fixture(params=[1, 0], ids=["critical_path", "level"])
def batch_order(request):
    """Plan with each work-item order (restored by _reset_options)."""
    qsim.set_option(qsim.OPT_BATCH_ORDER, request.param)
    return request.param


@pytest.mark.parametrize("kmax", [5, 6])
@pytest.mark.parametrize("fold", [1, 0])
def test_batch_folded_start(fold, kmax):
    """The uniform start written together with each circuit's first cluster
    (one write-only op: w over the cluster's targets times the column's
    epilogue factor) or as a separate initialisation; both against the oracle."""
    qsim.set_option(qsim.OPT_FOLD_INIT, fold)
    circs = small_batch(10, seed0=120 + kmax)
    b = qsim.Batch(circs, kmax=kmax)
    st = b.run()
    # ops: one initialisation per circuit unless folded
    n_sched = sum(len(qsim.schedule(c.n, c.gates, kmax=kmax, fuse_diag=True, skip_initial_h=True)["op_kind"])
                  for c in circs)
    assert st["n_ops"] == n_sched + (0 if fold else len(circs))
    check_against_oracle(b, circs)


@pytest.mark.parametrize("opts", [
    dict(),
    dict(fuse_diag=False),
    dict(kmax=3),
    dict(kmax=1, fuse_diag=False, skip_initial_h=False),
    dict(kmax=4, skip_initial_h=False),
    dict(kmax=6),
    dict(kmax=6, fuse_diag=False),
    dict(kmax=6, skip_initial_h=False),
])
def test_batch_matches_oracle(opts, batch_order):
    circs = small_batch(12, seed0=3)
    b = qsim.Batch(circs, **opts)
    st = b.run()
    assert st["n_circuits"] == 12 and st["n_items"] > 0
    check_against_oracle(b, circs)


@pytest.mark.parametrize("grid", [1, 3, 64])
def test_batch_any_grid(grid, batch_order):
    """One work-group runs every item in ticket order; a few work-groups
    wait on each other; results do not depend on the grid."""
    qsim.set_option(qsim.OPT_BATCH_GRID, grid)
    circs = small_batch(6, seed0=40)
    b = qsim.Batch(circs)
    st = b.run()
    assert st["grid"] == min(grid, st["n_items"])
    check_against_oracle(b, circs)


def test_batch_high_padding():
    qsim.set_option(qsim.OPT_BATCH_PAD, 1)
    circs = small_batch(6, seed0=60)
    b = qsim.Batch(circs, kmax=3)
    b.run()
    check_against_oracle(b, circs)


def test_batch_dense_gates_and_skips():
    """Haar 5- and 3-qubit gates inside the circuits; trailing diagonal gates skipped."""
    circs = []
    for i, n in enumerate((12, 14, 15, 11)):
        R, C, drop = batch_grid(n)
        c = supremacy_circuit(R, C, 20 + 3 * i, 500 + i, drop)
        circs.append(with_haar_layers(c, 6, 5 if i % 2 == 0 else 3, 900 + i))
    b = qsim.Batch(circs, skip_trailing_diag=True)
    b.run()
    check_against_oracle(b, circs, skip_trailing_diag=True)
    b2 = qsim.Batch(circs)
    b2.run()
    check_against_oracle(b2, circs)


@pytest.mark.parametrize("pad", [0, 1])
def test_batch_six_qubit_clusters(pad):
    """6-qubit clusters (fp16 matrix halves, staged half tiles) next to padded
    smaller ones in one launch: Haar 6-qubit gates, targets on the lowest
    qubits and elsewhere, qubit 0 a target or not."""
    qsim.set_option(qsim.OPT_BATCH_PAD, pad)
    circs = []
    for i, n in enumerate((11, 12, 14, 16, 13)):
        R, C, drop = batch_grid(n)
        c = supremacy_circuit(R, C, 14 + 4 * i, 700 + i, drop)
        circs.append(with_haar_layers(c, 5, 6, 950 + i))
    scheds = [qsim.schedule(c.n, c.gates, kmax=6, fuse_diag=True, skip_initial_h=True) for c in circs]
    assert any(6 in s["op_k"] for s in scheds) and any(k < 6 for s in scheds for k in s["op_k"])
    b = qsim.Batch(circs, kmax=6)
    b.run()
    check_against_oracle(b, circs)


def test_batch_repeat_runs_and_two_batches():
    circs = small_batch(5, seed0=80)
    b = qsim.Batch(circs)
    b.run()
    first = [s.cpu().numpy() for s in b.states]
    b.run()
    for s, f in zip(b.states, first):
        assert np.array_equal(s.cpu().numpy(), f)
    other = small_batch(3, n_lo=12, n_hi=13, seed0=90)
    b2 = qsim.Batch(other)
    b2.run()
    check_against_oracle(b2, other)
    check_against_oracle(b, circs)


def test_batch_single_circuit_sizes():
    """The smallest state (one tile), a ragged mix, and a 20-qubit state."""
    for n, depth in ((11, 12), (20, 25)):
        R, C, drop = batch_grid(n)
        circ = supremacy_circuit(R, C, depth, 7 + n, drop)
        b = qsim.Batch([circ])
        b.run()
        check_against_oracle(b, [circ])


def test_batch_wait_limit_reports_error():
    """A wait forced to give up (a 1 us limit, set by the host: the items of
    the 20-qubit initialisation take far longer) is reported; the kernel
    still exits and the next run with the default limit is exact."""
    circ = supremacy_circuit(4, 5, 16, 3)
    b = qsim.Batch([circ])
    with pytest.raises(qsim.QsimError) as ei:
        b.run(wait_limit_us=1)
    assert ei.value.status == qsim.E_DEVICE
    b.run()
    check_against_oracle(b, [circ])


def test_batch_full_size_sample():
    """The 512-circuit workload (n in [14, 24], depth in [10, 40], seeds
    1000 + i) in one launch. Every circuit is compared with the library's
    float64 per-gate path (itself held to the oracle at 1e-12), and a seeded
    subset of 64 - every 8th circuit, indices 0, 8, ..., 504, all sizes from
    14 to 24 qubits - with the oracle directly."""
    import torch
    circs = [batch_circuit(i) for i in range(512)]
    b = qsim.Batch(circs)
    st = b.run()
    assert st["n_circuits"] == 512
    worst = 1.0
    for i, c in enumerate(circs):
        s = qsim.State(c.n, "c128")
        s.run_circuit(c.gates, scheduler="per_gate")
        f, _ = s.compare(b.states[i].to(torch.complex128))
        worst = min(worst, f)
        del s
    assert worst >= 1 - 1e-6, worst
    subset = list(range(0, 512, 8))
    assert sorted({circs[i].n for i in subset}) == list(range(14, 25))
    check_against_oracle(b, [circs[i] for i in subset], index=subset)
