import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def paper():
    with open(os.path.join(GOLDEN, "paper_values.json")) as f:
        return json.load(f)


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def tab32(orc):
    """Oracle checkpoints of U(r) over the whole 32-bit skip period."""
    p, a = orc.lcg_params(32)
    return orc.SkipTab(p, a, 1 << 16, p - 1)


@pytest.fixture(scope="session")
def tab64(orc):
    """Oracle checkpoints of U(r) for the 64-bit skip up to r = 2^28."""
    p, a = orc.lcg_params(64)
    return orc.SkipTab(p, a, 1 << 16, (1 << 28) - 1)
