import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def read_golden(name):
    """Parse a golden fixture: '#' lines are comments, other lines are
    'key: v1 v2 ...' with integer or float values."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, _, rest = line.partition(":")
            vals = []
            for tok in rest.split():
                try:
                    vals.append(int(tok, 0))
                except ValueError:
                    vals.append(float(tok))
            out[key.strip()] = vals
    return out


@pytest.fixture
def golden():
    return read_golden
