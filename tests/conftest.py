import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU; runs the HIP path")
    config.addinivalue_line("markers", "slow: long CPU test")


_GPU = None


def _gpu_available():
    global _GPU
    if _GPU is None:
        try:
            import torch
            _GPU = bool(torch.cuda.is_available())
        except Exception:
            _GPU = False
    return _GPU


def pytest_runtest_setup(item):
    if "gpu" in item.keywords and not _gpu_available():
        pytest.skip("no GPU in this environment")
