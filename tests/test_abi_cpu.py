"""The C-ABI library loads without a GPU and exports every symbol its header
declares; host-only argument checks work."""
import ctypes
import os
import re

import numpy as np
import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "qsim.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qsim_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("qsim_create", "qsim_apply_cluster", "qsim_apply_diag", "qsim_run_circuit",
                     "qsim_probs"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1704_01127_amd import qsim
    lib = qsim.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_workspace_and_argument_errors_without_gpu():
    from paper_1704_01127_amd import qsim
    L = qsim.lib()
    assert qsim.workspace_bytes(30, qsim.C64, 5) < qsim.workspace_bytes(30, qsim.C128, 6)
    h = ctypes.c_void_p()
    # null buffers / bad n are rejected on the host before any GPU call
    assert L.qsim_create(30, qsim.C64, None, 0, None, 0, None, 0, ctypes.byref(h)) == -1
    assert L.qsim_create(40, qsim.C64, ctypes.c_void_p(256), 1 << 40, ctypes.c_void_p(256),
                         1 << 30, None, 0, ctypes.byref(h)) == -2
    assert b"n_qubits" in L.qsim_last_error()
    assert L.qsim_apply_cluster(None, 1, None, None) == -1


def test_schedule_rejects_bad_gates():
    from paper_1704_01127_amd import qsim
    with pytest.raises(qsim.QsimError, match="out of range"):
        qsim.schedule(4, [("H", (4,))])
    with pytest.raises(qsim.QsimError, match="repeated"):
        qsim.schedule(4, [("CZ", (1, 1))])
    with pytest.raises(qsim.QsimError, match="kmax"):
        qsim.schedule(4, [("H", (0,))], kmax=8)
    with pytest.raises(ValueError, match="at most 6"):
        qsim.gate_array([("U", tuple(range(7)), np.eye(128, dtype=np.complex128))])
    # the library's own check: a dense gate of 7 qubits is refused
    arr, keep = qsim.gate_array([("U", tuple(range(6)), np.eye(64, dtype=np.complex128))])
    arr[0].k = 7
    nops = ctypes.c_int()
    o = qsim.run_opts(kmax=7)
    cap = 4
    i32 = lambda m: (ctypes.c_int32 * m)()
    assert qsim.lib().qsim_schedule(8, arr, 1, ctypes.byref(o), i32(1), i32(1), i32(cap), i32(cap),
                                    i32(cap * qsim.MAX_CLUSTER), cap, ctypes.byref(nops)) == qsim.E_UNSUPPORTED
    assert b"dense gates" in qsim.lib().qsim_last_error()


def test_seven_qubit_cap():
    """kmax = 7 forms 7-qubit clusters only where a kernel exists for them:
    complex64 states of >= 12 qubits with the fp16-halves 6-qubit kernel;
    elsewhere schedules are capped at 6 qubits."""
    from paper_1704_01127_amd import qsim
    from supremacy_inputs import supremacy_circuit
    circ = supremacy_circuit(5, 6, 25, 0)

    def widest(n=circ.n, gates=circ.gates, dtype=qsim.C64):
        sch = qsim.schedule(n, gates, dtype=dtype, kmax=7, fuse_diag=True, skip_initial_h=True,
                            skip_trailing_diag=True)
        return max(k for k, kind in zip(sch["op_k"], sch["op_kind"]) if kind == 0)

    assert widest() == 7
    assert widest(dtype=qsim.C128) == 6
    small = supremacy_circuit(3, 3, 20, 0)  # 9 qubits
    assert widest(small.n, small.gates) <= 6
    old = qsim.get_option(qsim.OPT_K6_KERNEL)
    try:
        qsim.set_option(qsim.OPT_K6_KERNEL, 0)
        assert widest() == 6
    finally:
        qsim.set_option(qsim.OPT_K6_KERNEL, old)


def test_batch_plan_host_checks():
    """Batch planning is host-only: its argument checks and workspace sizing
    run without a GPU (the amplitude pointers are never dereferenced)."""
    import ctypes
    from paper_1704_01127_amd import qsim
    from supremacy_inputs import supremacy_circuit
    L = qsim.lib()
    circ = supremacy_circuit(3, 4, 12, 1)
    ga, keep = qsim.gate_array(circ.gates)

    def plan(n=12, ptrs=(1 << 20, 2 << 20), **opts):
        arr = (qsim.BatchCircuit * len(ptrs))()
        for i, p in enumerate(ptrs):
            arr[i].n_qubits = n
            arr[i].n_gates = len(circ.gates)
            arr[i].gates = ctypes.cast(ga, ctypes.POINTER(qsim.Gate))
            arr[i].dev_amps = p
        o = qsim.run_opts(**dict(dict(kmax=5, fuse_diag=True), **opts))
        h, ws = ctypes.c_void_p(), ctypes.c_size_t()
        st = L.qsim_batch_plan(arr, len(ptrs), ctypes.byref(o), ctypes.byref(h), ctypes.byref(ws))
        if st == 0:
            L.qsim_batch_destroy(h)
        return st, ws.value

    st, ws = plan()
    assert st == 0 and ws > 2 * 16384
    st2, ws2 = plan(fuse_diag=False)
    assert st2 == 0 and ws2 >= ws  # diagonal passes become extra cluster ops
    st6, ws6 = plan(kmax=6)
    assert st6 == 0 and ws6 > 0                     # 6-qubit clusters: fp16 matrix halves (64 KiB each)
    assert plan(kmax=7)[0] == qsim.E_UNSUPPORTED
    assert plan(scheduler="per_gate")[0] == qsim.E_UNSUPPORTED
    assert plan(n=10)[0] == qsim.E_UNSUPPORTED      # below one tile
    assert plan(ptrs=(1 << 20, 1 << 20))[0] == qsim.E_INVALID  # shared state
    assert plan(ptrs=(1 << 20, (2 << 20) + 8))[0] == qsim.E_INVALID  # unaligned
    assert plan(n=11)[0] == qsim.E_INVALID          # the circuit's qubit 11 is out of range
    assert L.qsim_batch_run(None, None, 0, None, 0, None) == qsim.E_INVALID


def test_unitarity_check_option():
    """QSIM_OPT_CHECK_UNITARY: dense matrices are checked on the host before
    anything runs (the schedule call is host-only)."""
    import numpy as np

    from paper_1704_01127_amd import qsim
    from supremacy_inputs import haar_unitary
    u = haar_unitary(3, 5)
    bad = u.copy()
    bad[0, 0] += 1e-6
    assert qsim.get_option(qsim.OPT_CHECK_UNITARY) == 0
    qsim.schedule(4, [("U", (0, 1, 3), bad)])  # off by default: accepted
    qsim.set_option(qsim.OPT_CHECK_UNITARY, 1)
    try:
        qsim.schedule(4, [("U", (0, 1, 3), u)])
        with pytest.raises(qsim.QsimError, match="not unitary"):
            qsim.schedule(4, [("H", (0,)), ("U", (0, 1, 3), bad)])
        with pytest.raises(qsim.QsimError, match="not unitary"):
            qsim.stage_schedule(4, [("U", (0, 1), 2 * np.eye(4, dtype=np.complex128))], 3)
    finally:
        qsim.set_option(qsim.OPT_CHECK_UNITARY, 0)
    with pytest.raises(qsim.QsimError):
        qsim.set_option(qsim.OPT_CHECK_UNITARY, 2)
