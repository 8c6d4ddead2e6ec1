import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_addoption(parser):
    parser.addoption("--runslow", action="store_true", default=False,
                     help="also run the tests marked slow (whole oracle solves at 32^4 and 48^3x8, minutes each)")


def pytest_collection_modifyitems(config, items):
    if config.getoption("--runslow") or os.environ.get("GF_RUN_SLOW") == "1":
        return
    skip = pytest.mark.skip(reason="slow oracle re-check: run with --runslow (or GF_RUN_SLOW=1)")
    for item in items:
        if "slow" in item.keywords:
            item.add_marker(skip)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: oracle runs that take more than a few seconds")


@pytest.fixture(scope="session")
def repo_root():
    return ROOT
