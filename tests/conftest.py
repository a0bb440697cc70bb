import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device)")
    config.addinivalue_line("markers", "slow: takes tens of seconds on the CPU")


def load_rock_table():
    """Layer rows of the paper's rock-property table, SI units (m^2/s^2)."""
    rows = []
    with open(os.path.join(ROOT, "tests", "golden", "rock_table.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [float(x) for x in line.split()]
            rows.append(v[1:])
    return np.array(rows)


def load_kv(name):
    out = {}
    with open(os.path.join(ROOT, "tests", "golden", name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split()
            out[k] = float(v)
    return out


@pytest.fixture(scope="session")
def rock_table():
    return load_rock_table()


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle
