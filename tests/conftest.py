import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) HIP device")


def pytest_collection_modifyitems(config, items):
    # GPU tests fail loudly (never skip) when the device or the library is
    # missing; only their selection is controlled with -m gpu / -m "not gpu".
    pass


@pytest.fixture(scope="session")
def repo_root():
    return ROOT


@pytest.fixture(scope="session")
def ctx():
    """A libdcgs context on cuda:0.  GPU tests fail (never skip) when the
    device or the library is missing."""
    import torch

    from paper_2511_23030_amd import dcgs
    assert torch.cuda.is_available(), "GPU test run without a visible HIP device"
    dcgs.lib()
    c = dcgs.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()
