import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def gpu():
    """The HIP library on a GPU; skips without a GPU, fails if the library is missing there."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU in this environment")
    from paper_1812_05401_amd import binding
    binding.load()
    torch.cuda.init()
    return binding
