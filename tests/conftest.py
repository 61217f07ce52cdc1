import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Under pytest-xdist every worker loads its own copy of the oracle, whose OpenMP loops would
# each start one spinning thread per core: the workers then oversubscribe the cores and run
# many times slower.  Share the cores among them (before any test loads the oracle).
if "PYTEST_XDIST_WORKER" in os.environ and "OMP_NUM_THREADS" not in os.environ:
    _workers = max(1, int(os.environ.get("PYTEST_XDIST_WORKER_COUNT", "1") or 1))
    os.environ["OMP_NUM_THREADS"] = str(max(1, (os.cpu_count() or 1) // _workers))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def O():
    """The CPU oracle (built on first use if the shared object is missing or stale)."""
    from oracle import oracle
    oracle.lib()
    return oracle
