import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI)")
    config.addinivalue_line("markers", "slow: longer CPU statistics")


@pytest.fixture(scope="session")
def orc():
    from oracle import oracle
    lib = os.environ.get("MCRT_ORACLE_LIB")
    if lib:
        # a separately built oracle (the sanitizer run sets this)
        oracle.use_library(lib)
    else:
        oracle.build(force=False)
    return oracle
