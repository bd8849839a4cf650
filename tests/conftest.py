import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Under pytest-xdist the oracle's OpenMP threads are shared out among the workers:
# every worker taking all host threads oversubscribes the host, and the spinning
# barriers of the small boxes then run a thousand times slower.
_workers = os.environ.get("PYTEST_XDIST_WORKER_COUNT", "")
if _workers.isdigit() and int(_workers) > 1 and "OMP_NUM_THREADS" not in os.environ:
    os.environ["OMP_NUM_THREADS"] = str(max(1, len(os.sched_getaffinity(0)) // int(_workers)))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: long CPU-side oracle runs")


@pytest.fixture(scope="session")
def orc():
    import oracle

    oracle.build(force=False)
    return oracle
