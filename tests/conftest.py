import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI)")
    config.addinivalue_line("markers", "slow: long-running CPU check")


@pytest.fixture(scope="session")
def cube1():
    """Unit cube, 4 x 4 x 2 triangles per face (192 triangles, 98 vertices)."""
    from synthetic import cube
    return cube(4)


@pytest.fixture(scope="session")
def c1_oracle(cube1):
    """Oracle blocks of the 192-triangle cube, 16 steps on (0, 1], alpha = 1."""
    import oracle
    v, t = cube1
    V, K = oracle.assemble(v, t, 1.0, 1.0, 16)
    return V, K
