import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# The oracle works on small dense matrices (d <= a few hundred), where a
# multi-threaded BLAS is many times slower than one thread: run it on one.
import numpy  # noqa: E402
import scipy.linalg  # noqa: E402,F401
from threadpoolctl import threadpool_limits  # noqa: E402

_BLAS_LIMIT = threadpool_limits(limits=1)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")
