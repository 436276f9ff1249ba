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
def orc():
    import oracle
    oracle.lib()
    return oracle


# Alternate builds for the sanitizer runs (tests/test_sanitizers.py): the
# parent test points these at instrumented copies of the two libraries.
if os.environ.get("BP_TEST_ORACLE_LIB"):
    import oracle as _oracle
    _oracle._LIB_PATH = os.environ["BP_TEST_ORACLE_LIB"]
if os.environ.get("BP_TEST_LIBRARY"):
    from paper_1902_09733_amd import _abi as _abi_mod
    _abi_mod.LIB_PATH = os.environ["BP_TEST_LIBRARY"]
