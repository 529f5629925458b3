import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device)")
    config.addinivalue_line("markers", "slow: long-running CPU check")


@pytest.fixture(scope="session")
def gpu_lib():
    """The built HIP library through its Python binding, on cuda:0."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_16103_amd import nanogs
    nanogs.load()
    return nanogs
