import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


# The autotuner's cache of a test session lives in a fresh temporary file, so that no choice
# timed elsewhere (a user's ~/.cache) decides which kernel variants the tests run.
if "MFWF_TUNE_CACHE" not in os.environ:
    import tempfile
    os.environ["MFWF_TUNE_CACHE"] = os.path.join(tempfile.mkdtemp(prefix="mfwf_tune_"), "tune.txt")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")
