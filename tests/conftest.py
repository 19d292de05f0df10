import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built libgpjc")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library, loaded through the Python binding.  GPU tests fail
    loudly if it is missing or no GPU is visible."""
    from paper_2601_05418_amd import gpjc
    return gpjc.load()
