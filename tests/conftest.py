import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running parity case")


@pytest.fixture(scope="session")
def gd():
    """The HIP binding; GPU tests only."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1310_0041_amd as m

    m.load()  # raises if the HIP library is missing
    return m
