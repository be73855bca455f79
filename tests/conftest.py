import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: full-size CPU work (minutes)")


@pytest.fixture(scope="session", autouse=True)
def _built_host_libs():
    """Build the generator and oracle shared objects once if absent."""
    import graphgen
    import oracle
    if not os.path.exists(graphgen._LIB_PATH):
        graphgen.build_lib()
    if not os.path.exists(oracle._LIB_PATH):
        oracle.build_lib()
