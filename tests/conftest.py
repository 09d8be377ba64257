import multiprocessing
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
TESTS = os.path.dirname(os.path.abspath(__file__))
if TESTS not in sys.path:
    sys.path.insert(0, TESTS)

# worker processes for the FP64 oracle in the full-size GPU tests (at most the CPU share of
# one GPU host)
MAX_ORACLE_WORKERS = 16


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def golden_dir():
    return os.path.join(ROOT, "tests", "golden")


_POOL = {"pool": None}


def _worker_init():
    # one BLAS thread per worker process (the library was loaded before the fork, so the
    # environment variables alone would come too late): the workers already fill the cores
    for v in ("OMP_NUM_THREADS", "MKL_NUM_THREADS", "OPENBLAS_NUM_THREADS"):
        os.environ[v] = "1"
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass


@pytest.fixture(scope="session", autouse=True)
def _oracle_pool_before_gpu(request):
    """Fork the oracle's worker processes at the start of a session that runs full-size GPU
    tests, before any test initialises the GPU, so that no worker inherits GPU state."""
    wanted = any(item.get_closest_marker("gpu") is not None and "fullsize" in item.nodeid
                 for item in request.session.items)
    if wanted:
        cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
        n = max(1, min(MAX_ORACLE_WORKERS, cores or 1))
        _POOL["pool"] = multiprocessing.get_context("fork").Pool(n, initializer=_worker_init)
    yield
    if _POOL["pool"] is not None:
        _POOL["pool"].terminate()
        _POOL["pool"].join()
        _POOL["pool"] = None


@pytest.fixture(scope="session")
def oracle_pool():
    if _POOL["pool"] is None:
        pytest.skip("oracle pool not started (run the full-size tests in their own session)")
    return _POOL["pool"]
