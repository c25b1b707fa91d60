"""pytest configuration: the `gpu` marker and import paths."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TESTS = os.path.dirname(os.path.abspath(__file__))
for p in (ROOT, TESTS):
    if p not in sys.path:
        sys.path.insert(0, p)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU run, skipped unless CLS_SLOW=1")


def pytest_collection_modifyitems(config, items):
    if os.environ.get("CLS_SLOW") == "1":
        return
    skip = pytest.mark.skip(reason="slow CPU test; set CLS_SLOW=1")
    for it in items:
        if "slow" in it.keywords:
            it.add_marker(skip)
