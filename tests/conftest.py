import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle import oracle as O

    O.lib()
    return O


@pytest.fixture(scope="session")
def fsne_lib():
    """The HIP library's binding (built in-tree first if it is missing)."""
    from paper_2509_07681_amd import fsne as F

    if not os.path.exists(F.LIB_PATH):
        from paper_2509_07681_amd.build import build

        build()
    F.load_library()
    return F
