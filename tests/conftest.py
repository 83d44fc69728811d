import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# hardware queues for the thirteen concurrent launches of the EM
# phase, read when the HIP runtime starts (before any test touches the GPU)
if int(os.environ.get("GPU_MAX_HW_QUEUES") or 0) < 13:
    os.environ["GPU_MAX_HW_QUEUES"] = "16"
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")
