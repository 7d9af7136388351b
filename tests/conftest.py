import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def rel_err(a, b):
    """Normwise relative l2 error ||a - b|| / ||b||."""
    import numpy as np
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b.ravel())
    if nb == 0:
        return float(np.linalg.norm(a.ravel()))
    return float(np.linalg.norm((a - b).ravel()) / nb)


@pytest.fixture(scope="session")
def gpu_lib():
    """The built HIP library on a machine with a GPU; skips otherwise."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_17867_amd import fmm
    return fmm
