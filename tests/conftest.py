import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def orc():
    """The FP64 CPU oracle (builds liboracle.so if it is not there yet)."""
    from oracle import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def tc():
    """The HIP library's Python binding; a GPU test without a GPU fails."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_1504_06289_amd as tc
    return tc
