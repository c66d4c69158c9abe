import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: oracle test that takes more than ~20 s")


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def sphere_c1():
    """Config-1 surface: unit sphere, 24 patches of 8x8 nodes (1,536 points)."""
    import synth
    return synth.cube_sphere(2, 8, 1.0)
