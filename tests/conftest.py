import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a HIP GPU (MI355X); runs the library through its C ABI")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle._load()
    return oracle


@pytest.fixture(scope="session")
def sfg():
    """The GPU binding; fails loudly if the library or the GPU is missing."""
    import torch
    from paper_1003_3684_amd import native
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    native.load()
    return native
