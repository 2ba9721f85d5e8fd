import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (runs the HIP library on the device)")
    config.addinivalue_line(
        "markers", "slow: long CPU test (physics validation of the oracle)")


def rel_l2(a, b):
    import numpy as np
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.linalg.norm(b.ravel())
    num = np.linalg.norm((a - b).ravel())
    if den == 0.0:
        return float(num)
    return float(num / den)


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle import build
    if not os.path.exists(build.LIB):
        build.build()
    return build.LIB
