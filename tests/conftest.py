import os
import sys

# the oracle works on many tiny matrices: threaded BLAS only adds overhead there; its
# Jacobi SVD spreads a batch of blocks over OpenMP threads (at most 16: the host share
# of one GPU)
for _v in ("OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")
os.environ.setdefault("OMP_NUM_THREADS", str(max(1, min(16, os.cpu_count() or 1))))
# the hardware queue count the benchmark runs with: every scale stream (and batch class)
# then runs on a queue of its own, so the tests see the same concurrency
os.environ["GPU_MAX_HW_QUEUES"] = "16"

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: oracle runs that take more than a few seconds")


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def lib():
    """The product binding; on a machine with a GPU a missing library is an error, not a skip."""
    import paper_1507_08751_amd as msld
    msld.load()
    return msld
