import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:  # pragma: no cover
        return False


@pytest.fixture(scope="session")
def gpu():
    """The HIP library bound to cuda:0; skips when no GPU is visible."""
    if not gpu_available():
        pytest.skip("no GPU visible")
    from paper_2509_12138_amd import _lib
    _lib.load()  # raises if libgsmi.so is missing: no fallback exists
    return _lib
