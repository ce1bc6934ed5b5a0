import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")
    config.addinivalue_line("markers", "slow: long CPU reproduction of the paper's tables (run with --runslow)")


def pytest_addoption(parser):
    parser.addoption("--runslow", action="store_true", default=False, help="run slow paper-table reproductions")


def pytest_collection_modifyitems(config, items):
    if config.getoption("--runslow"):
        return
    skip = pytest.mark.skip(reason="slow paper-table reproduction; use --runslow")
    for item in items:
        if "slow" in item.keywords:
            item.add_marker(skip)
