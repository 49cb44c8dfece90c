import gc
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU oracle runs")


def pytest_collection_modifyitems(config, items):
    # GPU tests run in one process on one device; order them after the CPU tests.
    items.sort(key=lambda it: 1 if it.get_closest_marker("gpu") else 0)


@pytest.fixture(autouse=True)
def _collect_cycles():
    """Collect reference cycles (frames kept by exception tracebacks) after each
    test, while module-scoped contexts are still held by their fixtures."""
    yield
    gc.collect()
