import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: large inputs (full-size workloads)")


@pytest.fixture(scope="session")
def nd():
    """The HIP library binding; GPU tests only."""
    import paper_1905_09758_amd as lib
    lib.require_gpu()
    return lib


@pytest.fixture(scope="session")
def nd_host():
    """The HIP library binding for its host-only entry points (no device)."""
    import paper_1905_09758_amd as lib
    return lib
