import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="module")
def torch_cuda():
    """torch with a visible GPU (the GPU tests' entry fixture)."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch
