import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


# (dnum, log2 N, ell, batch) of the four benchmark parameter sets.
CONFIGS = {
    "d2-n13-l6": (2, 13, 6, 1),
    "d2-n15-l10": (2, 15, 10, 32),
    "d4-n16-l32": (4, 16, 32, 8),
    "d8-n17-l56": (8, 17, 56, 2),
}


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.lib()
    return oracle
