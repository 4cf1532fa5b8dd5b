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
    the file named by FV_PARITY_REPORT, when set (the tests also print them)."""
    path = os.environ.get("FV_PARITY_REPORT")
    if not path:
        return
    try:
        from tests import parity
    except Exception:
        return
    if not parity.REPORT:
        return
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as fh:
        fh.write("\n".join(parity.REPORT) + "\n")
