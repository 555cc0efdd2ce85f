import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running statistical test")


@pytest.fixture(scope="session")
def orc():
    from oracle import binding, build
    if not os.path.exists(binding.LIB_PATH):
        build.build()
    return binding


@pytest.fixture(scope="session")
def xs_default():
    from paper_2103_09642_amd.workloads import synthetic_xsec
    return synthetic_xsec()
