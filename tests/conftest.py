import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    import oracle
    oracle.load()
    yield


def pytest_collection_finish(session):
    # import torch during collection so the first GPU test does not pay for it
    if any(item.get_closest_marker("gpu") for item in session.items):
        import torch  # noqa: F401
