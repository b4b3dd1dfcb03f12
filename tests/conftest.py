import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library through the C ABI)")
    config.addinivalue_line("markers", "slow: long CPU-only oracle runs")


@pytest.fixture(scope="session")
def cuda():
    import torch
    # GPU tests run only where a GPU is expected: fail loudly instead of skipping
    assert torch.cuda.is_available(), "GPU test collected on a machine without a GPU"
    return torch.device("cuda:0")
