import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_sessionstart(session):
    # The oracle's many small BLAS calls run fastest on one thread (with one
    # thread per core they are ~20x slower).  threadpoolctl limits only the
    # libraries already loaded, so numpy and scipy are imported first.
    try:
        import numpy  # noqa: F401
        import scipy.linalg  # noqa: F401
        from threadpoolctl import threadpool_limits
        session._afq_blas_limit = threadpool_limits(1)
    except Exception:
        pass


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")
