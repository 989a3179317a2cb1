import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library and a visible GPU.  On a GPU run a missing library is
    an error, never a skip."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("gpu test collected but no GPU is visible")
    import paper_1410_2697_amd as mfh
    mfh.load()
    return mfh
