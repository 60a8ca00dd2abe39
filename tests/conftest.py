import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: full-size oracle runs (tens of seconds)")


def load_golden(name):
    path = os.path.join(ROOT, "tests", "golden", name)
    den = None
    rows = []
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line.startswith("# denominator"):
                den = float(line.split()[-1])
                continue
            if not line or line.startswith("#"):
                continue
            rows.append([float(x) for x in line.split()])
    import numpy as np
    return np.array(rows) / den
