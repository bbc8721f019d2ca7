import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds")
    # The oracle is plain C; build it once if nothing is built yet.
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        from oracle import build as _ob
        _ob.build()


@pytest.fixture(scope="session")
def gpu():
    """Skip-free GPU gate: GPU tests fail loudly if there is no GPU or no library."""
    import torch
    assert torch.cuda.is_available(), "GPU test run without a visible GPU"
    import paper_2601_00551_amd as sbp
    sbp.load()
    return torch.device("cuda:0")
