import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI)")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    from oracle import build
    if not os.path.exists(build.LIB):
        build.build()
    yield


@pytest.fixture(scope="session")
def threads():
    """Oracle threads for the heavier physics pins (results do not depend on it)."""
    from oracle.binding import set_threads
    n = max(1, min(8, os.cpu_count() or 1))
    set_threads(n)
    yield n
    set_threads(1)
