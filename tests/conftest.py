import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Scoring sets (match, mismatch, gap_open, gap_extend); a gap of length k
# scores gap_open + (k-1)*gap_extend.
CONFIG_SCORING = (1, -3, -5, -2)
SCORING_SETS = [
    CONFIG_SCORING,
    (1, -3, -7, -2),      # the same defaults under the q + k*r gap convention
    (2, -1, -3, -3),      # linear gaps
    (1, -1, -2, -1),
    (5, -4, -10, 0),      # free gap extension
    (1, -3, -5, -2 * 1),
]


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def pytest_collection_modifyitems(config, items):
    if gpu_available():
        return
    skip = pytest.mark.skip(reason="no GPU in this environment")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)
