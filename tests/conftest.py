import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library through its Python binding; skips nothing: a GPU test
    that cannot load the library fails loudly."""
    import torch  # noqa: F401  (loads the HIP runtime the library binds to)
    from paper_1812_06765_amd import ngf
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    return ngf
