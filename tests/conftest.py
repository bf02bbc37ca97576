import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_sessionstart(session):
    # The oracle's many small BLAS calls run fastest on one thread.
    try:
        from threadpoolctl import threadpool_limits
        session._afq_blas_limit = threadpool_limits(1)
    except Exception:
        pass


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")
