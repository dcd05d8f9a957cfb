import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def tables():
    from paper_1704_01202_amd import workloads as W
    return W.make_tables()


@pytest.fixture(scope="session")
def orc():
    from oracle import oracle as O
    O.lib()
    return O
