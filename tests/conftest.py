import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP scan library, loaded through its Python binding.

    GPU tests must run the native library: a missing build or a missing
    device is an error, never a silent fallback.
    """
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU test collected on a host without a GPU")
    from paper_1604_04815_amd import binding

    binding.load()
    return binding
