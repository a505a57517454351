import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~20 s")


@pytest.fixture(scope="session")
def sphere_small():
    """Icosphere nsub 2, radius 0.5 wavelength (480 RWG), dense oracle Z and dZ/dk."""
    import numpy as np
    import workloads
    from oracle import efie
    V, F = workloads.icosphere(2, 0.5)
    Z, dZ = efie.dense_Z(V, F, 2 * np.pi, deriv=True)
    return V, F, Z, dZ


@pytest.fixture(scope="session")
def sphere_cfg1():
    """Icosphere nsub 3, radius 0.5 wavelength (1,920 RWG), dense oracle Z."""
    import numpy as np
    import workloads
    from oracle import efie
    V, F = workloads.icosphere(3, 0.5)
    return V, F, efie.dense_Z(V, F, 2 * np.pi)
