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


@pytest.fixture(scope="session")
def adr():
    """The HIP binding, built first if the library is missing."""
    import importlib.util
    path = os.path.join(ROOT, "paper_2307_10684_amd", "build.py")
    spec = importlib.util.spec_from_file_location("_adr_build", path)
    _build = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(_build)   # by path: the package import needs the library
    if not os.path.exists(_build.LIB):
        _build.build()
    import paper_2307_10684_amd
    return paper_2307_10684_amd


@pytest.fixture(scope="session")
def dev(adr):
    """The GPU binding; fails (does not skip) when no GPU is visible."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X (select them with -m gpu)"
    return adr
