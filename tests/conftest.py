import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: large full-size parity case")


@pytest.fixture(scope="session")
def dfb_host():
    """The built C-ABI library, loaded for host-only calls (no GPU work)."""
    import paper_2305_07083_amd as m
    return m.load()
