import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.dirname(os.path.abspath(__file__))
for p in (ROOT, HERE):
    if p not in sys.path:
        sys.path.insert(0, p)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU-only oracle runs")


def golden_path(name):
    return os.path.join(HERE, "golden", name)


def pytest_collection_modifyitems(session, config, items):
    """Tests of the serving engine (a native engine thread per server) run
    after the other GPU tests and before the allocation-free entry point's
    test, which stays last; the order within each group is unchanged."""
    def rank(item):
        path = str(item.fspath)
        if os.path.basename(path).startswith("test_zz_"):
            return 2
        return 1 if os.path.basename(path) == "test_gpu_serve.py" else 0
    items[:] = sorted(items, key=rank)  # stable: keeps the order inside each rank
