import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line('markers', 'gpu: needs an MI355X (runs the HIP path)')


def golden(name):
    rows = []
    with open(os.path.join(ROOT, 'tests', 'golden', name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith('#'):
                rows.append([float(v) for v in line.split()])
    return rows
