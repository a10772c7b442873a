import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_addoption(parser):
    parser.addoption("--oracle-lib", default=None,
                     help="load the oracle from this build of oracle/*.c (e.g. the sanitizer build)")
    parser.addoption("--nnm-lib", default=None,
                     help="load libnnm from this build (e.g. the sanitizer build of the host code)")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU check")
    oracle_lib = config.getoption("--oracle-lib")
    if oracle_lib:
        from oracle.build import select_library
        select_library(oracle_lib)
    nnm_lib = config.getoption("--nnm-lib")
    if nnm_lib:
        import paper_2201_09147_amd as nnm
        nnm.load_library(nnm_lib)


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    """The oracle library is built by __graft_entry__.build(); build it here only if absent."""
    from oracle.build import build_oracle, oracle_lib_path
    if not os.path.exists(oracle_lib_path()):
        build_oracle()
    yield
