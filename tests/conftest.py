import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


GOLDEN = os.path.join(ROOT, "tests", "golden")


def read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


@pytest.fixture(autouse=True)
def _announce_gpu_case(request):
    """Print and flush the case name before each GPU test, so a run that dies
    on the device still names the case it was running."""
    if request.node.get_closest_marker("gpu") is not None:
        tr = request.config.pluginmanager.get_plugin("terminalreporter")
        if tr is not None:
            tr.write_line("[gpu case] %s" % request.node.nodeid, flush=True)
    yield


U32 = 2.0 ** -24


def fp32_circuit_bound(max_amp, n_ops, kmax):
    """Largest |d amp| allowed for a complex64 run of n_ops cluster passes
    (clusters of <= kmax qubits) against the float64 oracle.

    One pass computes every output as a dot product of 2^(kmax+1) real
    terms. Its rounding errors, of order u = 2^-24 relative each, add up like
    a random walk, to about sqrt(2^(kmax+1)) u times the output's scale,
    which is at most max|amp|; unitary passes do not amplify earlier errors,
    so n_ops passes add at most n_ops such terms. A factor 4 covers the
    rounding of the inputs and matrices. Arithmetic with fewer significant
    bits (plain fp16: u = 2^-11) exceeds this bound by orders of magnitude."""
    return 4.0 * n_ops * (2.0 ** (kmax + 1)) ** 0.5 * U32 * max_amp
