import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built libxf.so")
    config.addinivalue_line("markers", "slow: long CPU test")


def oracle_objects(case):
    """oracle Thermo and Grid for a workloads.Case"""
    import oracle as O
    th = O.Thermo(case.thermo.W, case.thermo.a, case.thermo.T_lo, case.thermo.T_hi)
    g = O.Grid(case.n[0], case.n[1], case.n[2], case.d[0], case.d[1], case.d[2], tuple(case.bc), case.ng)
    return th, g


@pytest.fixture
def rng():
    return np.random.default_rng(1234)
