import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built liblbm.so")
    config.addinivalue_line("markers", "slow: physics runs of the oracle that take several seconds")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    from oracle import build as ob
    if not os.path.exists(ob.LIB):
        ob.build(force=False)
    yield
