import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD GPU (MI355X) and the built HIP library")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    """Build the CPU oracle library once if it is not there yet."""
    from oracle.build import LIB, build
    if not os.path.exists(LIB):
        build()
    yield


TABLE1 = dict(sin2_th12=0.311, sin2_th23=0.5, sin2_th13=0.0251,
              dm2_32=2.4e-3, dm2_21=7.6e-5, delta_cp=0.0)
