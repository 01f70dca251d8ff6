"""Shared pytest configuration.

Tests marked `gpu` need an MI355X (gfx950) and the built HIP library; every
other test runs on the CPU.
"""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a gfx950 GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def pytest_collection_modifyitems(config, items):
    """Skip GPU tests when no GPU is visible (e.g. a plain CPU run)."""
    if not any(item.get_closest_marker("gpu") for item in items):
        return
    try:
        import torch
        have_gpu = torch.cuda.is_available()
    except Exception:
        have_gpu = False
    if have_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for item in items:
        if item.get_closest_marker("gpu"):
            item.add_marker(skip)
