import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU (select with -m gpu)")
    config.addinivalue_line("markers", "slow: oracle checks that take tens of seconds")


def results_dir():
    """Folder the study tests write their tables to (JSON), created on use;
    IBR_RESULTS_DIR overrides it."""
    out = os.environ.get("IBR_RESULTS_DIR", os.path.join(ROOT, "gpurun_out"))
    os.makedirs(out, exist_ok=True)
    return out


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def rng():
    import numpy as np
    return np.random.default_rng(1234)
