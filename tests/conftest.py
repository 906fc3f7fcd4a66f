import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# the library's autotuners keep their results in this file during the tests
# (read when the library first needs it), not in the user's cache
os.environ.setdefault("PGABB_TUNE_CACHE", "/tmp/pgabb_tune_tests_%d.txt" % os.getpid())


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (run with -m gpu)")
    config.addinivalue_line("markers", "slow: long CPU test")
