import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: oracle runs that take more than a few seconds")


def pytest_collection_modifyitems(config, items):
    # GPU tests fail loudly (not skip) when the device is missing but requested,
    # so that a silent CPU fallback can never pass them.
    pass
