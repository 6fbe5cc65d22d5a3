import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Parallel test workers (pytest-xdist) share the cores: each worker's OpenMP
# oracle gets its share, since several workers each spinning a full team at the
# oracle's per-step barriers slow every one of them by orders of magnitude. Set
# before anything loads the OpenMP runtime.
_WORKERS = int(os.environ.get("PYTEST_XDIST_WORKER_COUNT", "1") or 1)
if _WORKERS > 1 and "OMP_NUM_THREADS" not in os.environ:
    os.environ["OMP_NUM_THREADS"] = str(max(1, (os.cpu_count() or 1) // _WORKERS))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")
