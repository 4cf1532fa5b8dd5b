import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def orc():
    from oracle import oracle
    oracle.lib()
    return oracle


def pytest_sessionfinish(session, exitstatus):
    """GPU runs: every parity error the tests measured, with its case, goes to
    gpurun_out/parity_report.txt (the tests also print them)."""
    try:
        from tests import parity
    except Exception:
        return
    if not parity.REPORT:
        return
    out = os.path.join(ROOT, "gpurun_out")
    os.makedirs(out, exist_ok=True)
    with open(os.path.join(out, "parity_report.txt"), "w") as fh:
        fh.write("\n".join(parity.REPORT) + "\n")
