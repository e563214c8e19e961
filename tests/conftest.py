import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than ~10 s on the CPU")


def gpu_available() -> bool:
    try:
        import torch

        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def arc():
    """The HIP library binding; GPU tests fail loudly if it is missing."""
    if not gpu_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_1807_07094_amd import arc as _arc

    _arc.lib()  # raises if libarc.so is missing or does not load
    return _arc
