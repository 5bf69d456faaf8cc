import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def qx():
    """The HIP binding, on a machine with a GPU only; fails loudly if the library is missing."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1612_02750_amd as q

    q.load()  # raises if libqx.so is missing: no fallback
    return q
