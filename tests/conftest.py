import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: large CPU case")


@pytest.fixture(scope="session")
def golden():
    import json

    with open(os.path.join(GOLDEN, "paper_examples.json")) as f:
        return json.load(f)


@pytest.fixture(scope="session")
def built_lib():
    """Path of libbytestore.so, building it (and the generator) when absent."""
    from paper_2209_00220_amd import build as b

    if not os.path.exists(b.LIB):
        import __graft_entry__

        __graft_entry__.build()
    return b.LIB
