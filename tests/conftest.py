import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def oracle():
    from oracle import cref
    cref.build()
    return cref


@pytest.fixture(scope="session")
def gpu():
    """The HIP binding and a context on device 0.  On a machine without a GPU
    the gpu-marked tests are skipped; where a GPU exists, a missing library is
    an error (no fallback)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_1710_01839_amd import mpgemm
    ctx = mpgemm.Context(0)
    yield mpgemm, ctx
    torch.cuda.synchronize()
    ctx.close()
