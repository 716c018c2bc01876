import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def pytest_sessionstart(session):
    """Where a GPU is visible the native library must load.  The GPU test modules import the package
    with importorskip, so that a checkout without the build still collects on a CPU-only machine; on a
    GPU machine that would turn a missing library into skipped tests instead of failures.
    (device_count() does not initialise the GPU.)"""
    try:
        import torch
        ngpu = torch.cuda.device_count()
    except Exception:
        return
    if ngpu > 0:
        import paper_1211_1680_amd  # noqa: F401  (raises ImportError when the library is not built)
