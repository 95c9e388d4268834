import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def ba200():
    from paper_2412_20980_amd import inputs
    return inputs.ba200()


@pytest.fixture(scope="session")
def ba10k():
    from paper_2412_20980_amd import inputs
    return inputs.ba10k()


@pytest.fixture(scope="session")
def cl200k():
    from paper_2412_20980_amd import inputs
    return inputs.chung_lu_200k()
