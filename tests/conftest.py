import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")
    config.addinivalue_line("markers", "slow: long CPU run (oracle over many steps)")


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle import oracle as orc
    if not os.path.exists(orc.LIB_PATH):
        from oracle import build
        build.build()
    return orc.load()
