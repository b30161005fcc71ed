import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library through the C ABI)")
    config.addinivalue_line("markers", "slow: long CPU test")


GOLDEN = os.path.join(ROOT, "tests", "golden")


def read_golden(name):
    rows, notes = [], {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line:
                continue
            if line.startswith("#"):
                parts = line[1:].split()
                if len(parts) == 2:
                    try:
                        notes[parts[0]] = float(parts[1])
                    except ValueError:
                        pass
                continue
            rows.append(line.split())
    return rows, notes
