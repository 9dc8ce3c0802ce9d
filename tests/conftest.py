import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: longer CPU-only runs of the oracle")


@pytest.fixture(scope="session")
def oracle():
    from oracle import oracle as O
    if not (os.path.exists(O.LIB) and os.path.exists(O.LIB_COUNT)):
        O.build(force=False)
    return O
