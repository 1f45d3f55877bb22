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
