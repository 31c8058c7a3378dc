import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line(
        "markers", "slow: CPU test that takes more than a few seconds")
    config.addinivalue_line(
        "markers", "fullsize_oracle: compares with the oracle butterfly of "
        "a full-size workload (computed in worker processes)")


def pytest_collection_modifyitems(config, items):
    # Order: CPU tests first, then GPU tests, each keeping file order.
    items.sort(key=lambda it: 1 if it.get_closest_marker("gpu") else 0)


def pytest_collection_finish(session):
    # the full-size GPU tests compare all N entries with the oracle's
    # butterfly: start those oracle runs now, beside the other tests
    if session.config.option.collectonly:
        return
    if any(it.get_closest_marker("fullsize_oracle") for it in session.items):
        import _fullsize_oracle
        _fullsize_oracle.prefetch()


def pytest_sessionfinish(session, exitstatus):
    mod = sys.modules.get("_fullsize_oracle")
    if mod is not None:
        mod.shutdown()


@pytest.fixture(scope="session")
def golden_dir():
    return os.path.join(ROOT, "tests", "golden")
