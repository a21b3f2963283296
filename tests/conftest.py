import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: longer CPU test")


def ensure_library():
    """Path of the built HIP library; builds it from source only if absent."""
    from paper_2311_18737_amd import LIB_PATH

    if not os.path.exists(LIB_PATH):
        from paper_2311_18737_amd.build import build

        build(verbose=False)
    return LIB_PATH


@pytest.fixture(scope="session")
def ispl_lib():
    ensure_library()
    from paper_2311_18737_amd import load_library

    return load_library()
