import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU-only test")


@pytest.fixture(scope="session")
def gpu():
    """The GPU binding; fails (not skips) when the HIP library is missing on a machine with a GPU."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_1102_3094_amd as lam
    lam.load()  # raises if the built library is missing
    return lam
