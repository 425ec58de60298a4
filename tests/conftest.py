import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    import oracle
    src = oracle.SRC
    if not os.path.exists(oracle.LIB) or os.path.getmtime(oracle.LIB) < os.path.getmtime(src):
        oracle.build(force=True)
    yield
