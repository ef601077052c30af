import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs on the GPU box)")
    config.addinivalue_line("markers", "slow: long CPU test")


def golden(key):
    """Value and tolerance of ``key`` in tests/golden/paper_values.txt."""
    path = os.path.join(ROOT, "tests", "golden", "paper_values.txt")
    with open(path) as fh:
        for line in fh:
            line = line.split("--")[0].strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] == key:
                return float(parts[1]), float(parts[2])
    raise KeyError(key)
