import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU check")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    """The oracle library is built by __graft_entry__.build(); build it here only if absent."""
    from oracle.build import build_oracle, oracle_lib_path
    if not os.path.exists(oracle_lib_path()):
        build_oracle()
    yield
