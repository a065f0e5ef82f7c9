import os
import sys

import pytest

# Under pytest-xdist every worker loads the OpenMP oracle; one thread each
# keeps the workers from oversubscribing the cores (set before the library
# is loaded, which is when the OpenMP runtime reads it).
if "PYTEST_XDIST_WORKER" in os.environ:
    os.environ["OMP_NUM_THREADS"] = "1"

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU (runs the HIP library)")
    config.addinivalue_line("markers", "slow: longer CPU-only oracle runs")
