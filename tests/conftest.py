import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def lib():
    """The built HIP library (ctypes); GPU tests fail loudly without it."""
    from paper_2012_02430_amd import _lib

    return _lib.load()


@pytest.fixture(autouse=True)
def _announce_gpu_case(request):
    """Name the case on stdout (flushed) before a GPU test touches the device."""
    if request.node.get_closest_marker("gpu") is not None:
        print(f"\n[gpu case] {request.node.nodeid}", flush=True)
    yield
