"""The C-ABI library loads without a GPU and exports every symbol its header
declares; host-only argument checks work."""
import ctypes
import os
import re

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
        qsim.schedule(4, [("H", (0,))], kmax=7)
