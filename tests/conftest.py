import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds")


def _ensure_library():
    """Build libnsl.so in-tree if (and only if) nothing is built yet."""
    lib = os.path.join(ROOT, "paper_2210_13641_amd", "libnsl.so")
    if not os.path.exists(lib):
        from paper_2210_13641_amd import build
        build.build()
    return lib


@pytest.fixture(scope="session")
def nsl():
    _ensure_library()
    from paper_2210_13641_amd import nsl as mod
    return mod


@pytest.fixture(scope="session")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")
