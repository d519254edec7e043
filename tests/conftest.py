import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session", autouse=True)
def _torch_hip_context_first(request):
    """In a session with GPU tests, bring up PyTorch's HIP context before any
    test drives the library through ctypes.  PyTorch initialises lazily; its
    first CUDA call after 44 ctypes-only tests once reported "No HIP GPUs are
    available" on an MI355X machine (the tests that allocate through PyTorch then
    failed), while the same tests passed when PyTorch had been initialised
    first."""
    if any(item.get_closest_marker("gpu") for item in request.session.items):
        try:
            import torch
        except ImportError:
            torch = None
        if torch is not None and torch.cuda.is_available():
            torch.cuda.init()
            torch.zeros(1, device="cuda")
            torch.cuda.synchronize()
    yield
