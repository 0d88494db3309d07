import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_addoption(parser):
    parser.addoption("--run-slow", action="store_true", default=False,
                     help="also run the tests marked slow (CPU analyses of several minutes each)")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test, run only with --run-slow")


def pytest_collection_modifyitems(config, items):
    if config.getoption("--run-slow"):
        return
    skip = pytest.mark.skip(reason="slow (several minutes): run with --run-slow")
    for item in items:
        if "slow" in item.keywords:
            item.add_marker(skip)


_CACHE = {}


@pytest.fixture(scope="session")
def oracle_cache():
    """Session cache for oracle stencils (building them is the slow part)."""
    return _CACHE


def pytest_sessionstart(session):
    # build the library only when nothing is built yet
    lib = os.path.join(ROOT, "paper_2312_14789_amd", "libmlbm.so")
    if not os.path.exists(lib):
        from paper_2312_14789_amd.build import build

        build()
