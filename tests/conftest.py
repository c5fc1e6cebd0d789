import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def read_matrices(name):
    """Parse a golden file of named 8x8 integer matrices."""
    import numpy as np
    mats, cur, rows = {}, None, []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#")[0].strip()
        if not line:
            continue
        parts = line.split()
        if len(parts) == 1 and not parts[0].lstrip("-").isdigit():
            if cur:
                mats[cur] = np.array(rows, np.int64)
            cur, rows = parts[0], []
        else:
            rows.append([int(v) for v in parts])
    if cur:
        mats[cur] = np.array(rows, np.int64)
    return mats


def read_table(name):
    out = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#")[0].strip()
        if line:
            out.append(line.split())
    return out


@pytest.fixture(scope="session")
def paper_factors():
    return read_matrices("paper_factors.txt")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.lib()
    return oracle
