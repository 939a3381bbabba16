import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


def cvdot(a, b):
    """<a,b> = sum conj(a) b over all components."""
    return np.vdot(np.ravel(a), np.ravel(b))


def rel_l2(a, b):
    a = np.ravel(a)
    b = np.ravel(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="session")
def gauge44():
    from ksinputs import make_gauge
    return make_gauge((4, 4, 4, 4), 0.5, 11, keep_thin=True)


@pytest.fixture(scope="session")
def gauge8():
    from ksinputs import make_gauge, SEEDS
    return make_gauge((8, 8, 8, 8), 0.3, SEEDS["gauge"](1), keep_thin=True)
