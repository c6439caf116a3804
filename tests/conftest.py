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
def _library_built():
    # libsrmdp.so is built in-tree when it is missing or was built from other
    # sources (content hash); a current library is used as it is
    from paper_2407_21085_amd import build as B
    B.ensure_built(verbose=True)
    yield


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    import oracle
    # rebuilt when missing or older than its C source or header
    lib = oracle._LIB_PATH
    srcs = [oracle._SRC, os.path.splitext(oracle._SRC)[0] + ".h"]
    stale = not os.path.exists(lib) or any(os.path.getmtime(s) > os.path.getmtime(lib) for s in srcs)
    oracle.build(force=stale)
    yield
