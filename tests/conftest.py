import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the libmpf C ABI)")


@pytest.fixture(scope="session")
def small_cloud():
    """The plain-ACM workload cell: r = 0.3, h 0.02 -> 0.08, seed 1."""
    import nodecloud
    return nodecloud.config_cloud("acm_small")


@pytest.fixture(scope="session")
def small_stencils(small_cloud):
    import nodecloud
    return nodecloud.stencils(small_cloud.pos, 30)
