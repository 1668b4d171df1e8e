import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a HIP device (MI355X)")
    config.addinivalue_line("markers", "slow: long CPU-only check, skipped unless LWE_SLOW=1")


def pytest_collection_modifyitems(config, items):
    if os.environ.get("LWE_SLOW") == "1":
        return
    skip = pytest.mark.skip(reason="slow check; set LWE_SLOW=1")
    for it in items:
        if "slow" in it.keywords:
            it.add_marker(skip)


@pytest.fixture(scope="session")
def orc():
    import oracle

    oracle.build()
    return oracle


@pytest.fixture(scope="session")
def ctx():
    """A library context on device 0.  Fails (does not skip) when the HIP library or the
    device is missing: GPU tests must run the native path."""
    import paper_2606_01211_amd as L

    c = L.Context(0)
    yield c
    c.close()
