import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def load_golden(name):
    """Parse a tests/golden text fixture: '[name rows cols]' then integer rows."""
    out = {}
    cur, rows = None, []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("["):
                if cur is not None:
                    out[cur[0]] = np.array(rows, dtype=np.int64).reshape(cur[1], cur[2])
                parts = line.strip("[]").split()
                cur, rows = (parts[0], int(parts[1]), int(parts[2])), []
            else:
                rows.append([int(t) for t in line.split()])
    if cur is not None:
        out[cur[0]] = np.array(rows, dtype=np.int64).reshape(cur[1], cur[2])
    return out


@pytest.fixture(scope="session")
def golden_hand():
    return load_golden("hand_worked_m2_m3.txt")
