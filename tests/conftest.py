import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def blosum():
    from inputs import blosum62
    return blosum62()


@pytest.fixture(scope="session")
def gpu():
    """The GPU binding; fails (does not skip) when no GPU or no built library."""
    import torch
    assert torch.cuda.is_available(), "GPU test run without a visible GPU"
    import paper_2309_09609_amd as sw
    sw.load()          # raises if the HIP library is missing
    return sw
