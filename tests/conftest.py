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
def gpu_lib():
    """The HIP-backed binding; fails loudly if the library or the GPU is missing."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("gpu test selected but torch sees no GPU")
    import paper_2512_21909_amd as cdcc
    cdcc.require_gpu()
    return cdcc
