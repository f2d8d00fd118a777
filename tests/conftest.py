import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def _ensure_built():
    """Build the HIP library and the oracle only if nothing is built yet."""
    lib = os.path.join(ROOT, "paper_1103_1399_amd", "libqaa.so")
    if not os.path.exists(lib):
        import __graft_entry__
        __graft_entry__.build()
    import oracle
    oracle.build()


_ensure_built()


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def worked_example():
    with open(os.path.join(GOLDEN, "worked_example_3sat.json")) as f:
        return json.load(f)
