import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="module")
def ctx():
    """A library context on cuda:0 bound to torch's current stream."""
    import torch
    from paper_1909_10286_amd import bl
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = bl.Context(0)
    c.set_stream(torch.cuda.current_stream())
    yield c
    torch.cuda.synchronize()
    c.close()


@pytest.fixture(scope="session")
def pool():
    """Process pool running oracle candidate evaluations."""
    from .oracle_pool import OraclePool
    p = OraclePool()
    yield p
    p.close()
