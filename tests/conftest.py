import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built pdhot library")


@pytest.fixture(scope="session")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="session", autouse=True)
def _oracle_threads():
    """Under pytest-xdist every worker runs its own oracle: one thread each,
    so the workers do not oversubscribe the cores."""
    if os.environ.get("PYTEST_XDIST_WORKER"):
        import oracle
        oracle.set_threads(1)
    yield
