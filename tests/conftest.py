import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session", autouse=True)
def _built():
    """Build the oracle, and the HIP library only if nothing is built yet."""
    import oracle
    oracle.build(force=False)
    from paper_2304_04214_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        from paper_2304_04214_amd.build import build
        build()
    yield


@pytest.fixture
def mutation():
    """Plant a deliberate mistake in the oracle for the duration of a test."""
    import oracle

    def set_(k):
        oracle.set_mutation(k)
    yield set_
    oracle.set_mutation(0)
