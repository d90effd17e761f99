import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP kernels through the C ABI)")
    config.addinivalue_line("markers", "slow: CPU test taking more than a few seconds")


@pytest.fixture(scope="session")
def oracle():
    import oracle as O
    O.lib()
    return O


@pytest.fixture(scope="session")
def prnglib():
    """The product library (built on demand only when no build is present)."""
    from paper_1003_1898_amd import _capi
    if not os.path.exists(_capi.LIB_PATH):
        from paper_1003_1898_amd.build import build
        build()
    return _capi.lib()
