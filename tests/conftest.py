import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def gpu_lib():
    """The built HIP library, loaded through its Python binding.  GPU tests
    fail (not skip) when the library or the device is missing."""
    import torch
    assert torch.cuda.is_available(), "GPU test run without a visible GPU"
    import paper_2101_00585_amd as ups
    ups.load()
    return ups
