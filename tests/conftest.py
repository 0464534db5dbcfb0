import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: statistical test that runs for tens of seconds")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    from oracle import oracle as o
    if not os.path.exists(o.LIB_PATH):
        o.build()
    yield
