import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: longer CPU test (still part of the default CPU suite)")


@pytest.fixture(scope="session")
def hex16():
    from synthetic.mesh import planar_hex
    return planar_hex(16, 16, 1.0e4)


@pytest.fixture(scope="session")
def sphere3():
    from synthetic.mesh import icosahedral
    return icosahedral(3)
