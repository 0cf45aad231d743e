import os
import sys

# Small dense BLAS calls are slower with every core spinning; keep the oracle's
# BLAS at a few threads unless the caller chose otherwise.
os.environ.setdefault("OPENBLAS_NUM_THREADS", "4")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: oracle runs of more than a few seconds")
