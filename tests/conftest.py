"""Shared pytest set-up: repository root on sys.path, GPU marker handling."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) device and the built HIP library")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library through its ctypes binding; a GPU test fails (not skips)
    when the extension is missing, so a silent fallback can never pass."""
    from paper_2602_05900_amd import binding
    lib = binding.load()
    n = binding.device_count()
    if n < 1:
        pytest.fail("no HIP device visible to the library")
    return lib
