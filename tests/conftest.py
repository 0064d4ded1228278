import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running")


@pytest.fixture(scope="session")
def lib_built():
    """The built C-ABI library path, or skip when it was not built."""
    from paper_2110_15853_amd import _lib
    path = _lib.library_path()
    if not os.path.exists(path):
        pytest.skip("libttdft.so not built (run __graft_entry__.build())")
    return path
