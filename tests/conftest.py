import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running full-size case")


@pytest.fixture(scope="session")
def gpu_lib():
    """The built HIP library, loaded through the Python binding. GPU tests
    fail (not skip) when it is missing: no CPU path exists."""
    import torch
    assert torch.cuda.is_available(), "GPU test run without a visible GPU"
    from paper_2012_07620_amd import binding
    return binding.library()
