"""Shared pytest configuration.

Markers:
  gpu   -- needs an MI355X (runs the HIP library); deselect with -m "not gpu".
  slow  -- long CPU-only oracle pins; skipped unless --runslow is given.
"""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_addoption(parser):
    parser.addoption("--runslow", action="store_true", default=False,
                     help="run the long CPU oracle pins marked slow")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: test needs an MI355X GPU")
    config.addinivalue_line("markers", "slow: long CPU-only test, needs --runslow")


def pytest_collection_modifyitems(config, items):
    if config.getoption("--runslow"):
        return
    skip = pytest.mark.skip(reason="long oracle pin; run with --runslow")
    for item in items:
        if "slow" in item.keywords:
            item.add_marker(skip)
