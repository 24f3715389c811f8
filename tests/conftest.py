import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# The oracle's dense eigensolves run on OpenBLAS, whose spinning threads
# collapse when the cores are shared (pytest-xdist workers, other jobs): a
# 1536 x 1536 Hermitian eigensolve took 37 s on 8 threads beside one busy
# process against 0.45 s on 4.  Half the cores, at most 4, per test process.
try:
    from threadpoolctl import threadpool_limits

    _BLAS_LIMIT = threadpool_limits(limits=max(1, min(4, (os.cpu_count() or 2) // 2)), user_api="blas")
except ImportError:   # the limit is a speed measure only
    _BLAS_LIMIT = None


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")
