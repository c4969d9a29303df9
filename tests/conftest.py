import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library through its Python binding; the GPU tests need both."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2409_14309_amd as sns
    sns.load()  # raises if the shared library is missing
    return sns
