import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Under pytest-xdist each worker runs the OpenMP oracle (and the planted-mistake
# runs start oracle processes of their own): share the cores out between the
# workers instead of starting a full team in each, whose spinning threads
# slow the suite down many times over.  Set before the oracle library loads.
_workers = os.environ.get("PYTEST_XDIST_WORKER_COUNT")
if _workers and "OMP_NUM_THREADS" not in os.environ:
    os.environ["OMP_NUM_THREADS"] = str(max(1, (os.cpu_count() or 1) // int(_workers)))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def orc():
    from oracle import oracle
    oracle.lib()
    return oracle
