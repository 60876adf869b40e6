import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: large CPU work (mutant builds, big oracle runs)")


@pytest.fixture(scope="session")
def orc():
    import oracle

    return oracle.get()


def gpu_available() -> bool:
    try:
        import torch

        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def bandred():
    """The HIP binding; fails loudly (no fallback) if the library is missing."""
    import paper_1709_00302_amd as br

    if not gpu_available():
        pytest.fail("GPU test collected on a machine without a GPU")
    br.load()
    return br
