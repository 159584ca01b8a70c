import ctypes
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Keep freed large blocks mapped so repeated big numpy temporaries reuse pages
# instead of faulting fresh ones (first-touch faults are slow in sandboxes).
try:
    _libc = ctypes.CDLL("libc.so.6")
    _libc.mallopt(-3, 1 << 30)        # M_MMAP_THRESHOLD
    _libc.mallopt(-1, 2 ** 31 - 1)    # M_TRIM_THRESHOLD
except OSError:
    pass


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def lib():
    from paper_2207_14304_amd import argus
    return argus.load()
