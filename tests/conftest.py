"""Shared pytest configuration.

Markers
-------
gpu   needs a real MI355X (gfx950) and the built HIP library; run with ``-m gpu``.
slow  a CPU test that takes more than about a minute; runs only when the
      environment variable ``ADR_SLOW=1`` is set.
"""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test, enabled by ADR_SLOW=1")


def pytest_collection_modifyitems(config, items):
    if os.environ.get("ADR_SLOW") == "1":
        return
    skip = pytest.mark.skip(reason="slow test: set ADR_SLOW=1 to run")
    for item in items:
        if "slow" in item.keywords:
            item.add_marker(skip)
