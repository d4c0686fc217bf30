import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running check")


import pytest  # noqa: E402


@pytest.fixture(scope="session")
def ctx():
    """One library context on the current GPU for the whole session."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_10917_amd as bs
    c = bs.bs_ctx_create(torch.cuda.current_device())
    yield c
    torch.cuda.synchronize()
    c.close()
