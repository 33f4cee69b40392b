import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")
    config.addinivalue_line("markers", "slow: longer CPU-only oracle checks")


def pytest_collection_modifyitems(config, items):
    # GPU tests need a HIP device; fail loudly (not skip) if one was asked for
    # with -m gpu but the library is missing -- that is checked in the tests.
    pass
