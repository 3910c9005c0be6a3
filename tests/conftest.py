import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU-side work (large oracle runs)")


@pytest.fixture(scope="session")
def gpu_lib():
    """The built HIP library through its Python binding; skips when no GPU."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1511_05690_amd as mt

    mt.load_library()
    return mt
