import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU-only run")


def pytest_collection_modifyitems(config, items):
    # GPU tests need a visible device; without one they are skipped, not failed,
    # so that `-m "not gpu"` and plain runs on a CPU host stay green.
    try:
        import torch
        have_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover
        have_gpu = False
    if have_gpu:
        return
    mexpr = (config.getoption("-m") or "").replace(" ", "")
    if "gpu" in mexpr and "notgpu" not in mexpr:
        return  # GPU tests explicitly selected: let them fail loudly
    skip = pytest.mark.skip(reason="no GPU visible")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)
