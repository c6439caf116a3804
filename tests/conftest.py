import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    import oracle
    # rebuilt when missing or older than its C source or header
    lib = oracle._LIB_PATH
    srcs = [oracle._SRC, os.path.splitext(oracle._SRC)[0] + ".h"]
    stale = not os.path.exists(lib) or any(os.path.getmtime(s) > os.path.getmtime(lib) for s in srcs)
    oracle.build(force=stale)
    yield
