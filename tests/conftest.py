import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


def read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


@pytest.fixture(scope="session")
def fig4a():
    """(coords 0-based list of 3 uint32 arrays, values float32, dims)."""
    import numpy as np
    rows = read_golden("fig4a_coo.txt")
    c = np.array([[int(r[0]) - 1, int(r[1]) - 1, int(r[2]) - 1] for r in rows], dtype=np.uint32)
    v = np.array([float(r[3]) for r in rows], dtype=np.float32)
    return [np.ascontiguousarray(c[:, m]) for m in range(3)], v, (4, 4, 4)
