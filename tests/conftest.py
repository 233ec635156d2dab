import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP library on cuda:0)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~20 s")


_HIER = {}


@pytest.fixture(scope="session")
def hierarchy():
    """Session cache of oracle hierarchies keyed by a workload name."""
    from oracle.multigrid import Hierarchy

    def get(name, make):
        if name not in _HIER:
            _HIER[name] = Hierarchy(make())
        return _HIER[name]
    return get
