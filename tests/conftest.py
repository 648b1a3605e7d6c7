import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# a contraction whose GPU work does not finish within a minute fails its test
# with QTN_ETIMEOUT instead of blocking the run (read when libqtn first waits)
os.environ.setdefault("QTN_SYNC_TIMEOUT_S", "60")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU test")
