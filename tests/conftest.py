import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# BCH_PARITY_LOG=<path>: write the statistics of every parity comparison (tie
# ratios, trajectory and one-step errors) per test to that JSON file
_LOG_PATH = os.environ.get("BCH_PARITY_LOG")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")
    if _LOG_PATH:
        from tests import helpers
        helpers.PARITY_LOG = []


@pytest.fixture(autouse=True)
def _parity_log_mark(request):
    if _LOG_PATH:
        from tests import helpers
        n0 = len(helpers.PARITY_LOG)
        yield
        for rec in helpers.PARITY_LOG[n0:]:
            rec.setdefault("test", request.node.nodeid)
    else:
        yield


def pytest_sessionfinish(session, exitstatus):
    if _LOG_PATH:
        from tests import helpers
        os.makedirs(os.path.dirname(os.path.abspath(_LOG_PATH)), exist_ok=True)
        with open(_LOG_PATH, "w") as fh:
            json.dump(helpers.PARITY_LOG, fh, indent=1)
