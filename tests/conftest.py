import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a HIP device (MI355X); runs the library's kernels")
    config.addinivalue_line("markers", "slow: longer CPU runs of the oracle")


@pytest.fixture(scope="session")
def ora():
    """The CPU oracle (built with g++ if its shared object is missing)."""
    import oracle
    from oracle import oracle as _o
    if not (os.path.exists(_o._LIB) and os.path.exists(_o._LIB_FMA)):
        oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def W():
    from paper_2306_09760_amd import workloads
    return workloads
