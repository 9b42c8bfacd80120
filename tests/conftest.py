import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def gpu_lib():
    """The C-ABI library loaded through the Python binding, on cuda:0."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_11181_amd import lib

    return lib.get()
