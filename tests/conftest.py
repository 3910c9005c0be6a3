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


@pytest.fixture(scope="module")
def general_path(gpu_lib):
    """Products take the general path (planes, MFMA GEMM, sparse tail) even
    where the one-kernel small-product path would serve them."""
    old = gpu_lib.small_product_limit()
    gpu_lib.set_small_product_limit(0)
    yield gpu_lib
    gpu_lib.set_small_product_limit(old)
