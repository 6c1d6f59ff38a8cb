import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI library)")
    config.addinivalue_line("markers", "slow: takes longer than a few seconds on the CPU")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build()
    return oracle


def pytest_collection_modifyitems(config, items):
    # slow tests (minutes of CPU) run only when GSLIC_SLOW=1
    if os.environ.get("GSLIC_SLOW") == "1":
        return
    skip = pytest.mark.skip(reason="slow; set GSLIC_SLOW=1 to run")
    for it in items:
        if "slow" in it.keywords:
            it.add_marker(skip)
