import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    # autotuned plans in the tests read and write a tune cache of their own, not the user's
    if not os.environ.get("SBP_TUNE_CACHE"):
        import tempfile

        fd, path = tempfile.mkstemp(prefix="sbp_tune_tests_", suffix=".txt")
        os.close(fd)
        os.environ["SBP_TUNE_CACHE"] = path
        config._sbp_tune_cache = path
    config.addinivalue_line("markers", "gpu: needs an AMD MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_collection_modifyitems(config, items):
    # GPU tests need a visible device; on a GPU-less host they are skipped, not failed.
    try:
        import torch

        have_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover
        have_gpu = False
    if have_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)


def pytest_unconfigure(config):
    path = getattr(config, "_sbp_tune_cache", None)
    if path and os.path.exists(path):
        os.remove(path)
