import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: longer CPU checks")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library through its Python binding; skips when no device is present."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2411_03002_amd import binding
    return binding.load()
