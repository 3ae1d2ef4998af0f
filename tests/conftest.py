import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def gpu_available() -> bool:
    try:
        import torch
        return bool(torch.cuda.is_available())
    except Exception:
        return False


@pytest.fixture(scope="session")
def qf():
    """The HIP library binding (GPU tests only).  Fails loudly if it cannot be
    loaded on a GPU machine."""
    if not gpu_available():
        pytest.skip("no GPU")
    import paper_2306_08152_amd as pkg
    return pkg
