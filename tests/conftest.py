import os
import sys
import warnings

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")
    try:
        from scipy.integrate import IntegrationWarning
        warnings.filterwarnings("ignore", category=IntegrationWarning)
    except Exception:  # pragma: no cover
        pass


def ensure_library_built():
    """Build libctpd.so in-tree if it is missing (hipcc cross-compiles without a GPU)."""
    from paper_1609_06041_amd import build as B
    if not os.path.exists(B.LIB):
        B.build()
    return B.LIB


@pytest.fixture(scope="session")
def libctpd():
    ensure_library_built()
    from paper_1609_06041_amd import ctpd
    return ctpd.load()


@pytest.fixture(scope="session")
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_1609_06041_amd import ctpd
    ctpd.load()          # fails loudly when the HIP library is missing
    return torch.device("cuda:0")
