import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built libjumpmd.so")
    config.addinivalue_line("markers", "slow: long statistical run")


@pytest.fixture(autouse=True)
def _announce(request):
    # name the case before any GPU work so a dying box still reports it
    if request.node.get_closest_marker("gpu"):
        print(f"\n[case] {request.node.nodeid}", flush=True)
    yield
