import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: larger CPU oracle cases")


@pytest.fixture(scope="session")
def gpu():
    """The HIP library bound to cuda:0 (skips when no GPU is visible)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_1604_00617_amd as acr
    acr.load()          # raises if the built library is missing: no fallback
    return acr
