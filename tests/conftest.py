import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def pytest_collection_modifyitems(config, items):
    # run GPU tests in file order but after CPU tests of the same file set
    pass


@pytest.fixture(scope="session")
def lib():
    """The built GPU library (skips when no GPU is visible)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2407_19892_amd as g
    g.load()
    return g
