import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library on the device)")
    config.addinivalue_line("markers", "slow: oracle runs of tens of seconds")


def pytest_collection_modifyitems(config, items):
    # GPU tests are only meaningful on a box with a ROCm device; elsewhere they are skipped
    # explicitly (not silently passed) so the CPU suite stays green.
    have_gpu = False
    try:
        import torch
        have_gpu = torch.cuda.is_available()
    except Exception:
        pass
    if have_gpu:
        return
    skip = pytest.mark.skip(reason="no ROCm GPU in this environment")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)
