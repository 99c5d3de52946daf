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


# Achieved errors of the GPU-vs-oracle parity checks, printed as each check
# runs and listed again at the end of the session.
_PARITY = []


@pytest.fixture
def parity(request):
    """parity(quantity, achieved, bar): record the achieved error of one
    parity check, print it, and assert it is within its bar."""
    def record(quantity, achieved, bar):
        achieved = float(achieved)
        _PARITY.append((request.node.nodeid, quantity, achieved, float(bar)))
        print(f"[parity] {request.node.nodeid} {quantity}: {achieved:.3e} (bar {bar:.0e})", flush=True)
        assert achieved <= bar, f"{quantity}: {achieved:.3e} above the bar {bar:.0e}"
    return record


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    if not _PARITY:
        return
    terminalreporter.section("achieved errors, GPU vs FP64 oracle (achieved <= bar)")
    for nodeid, quantity, achieved, bar in _PARITY:
        terminalreporter.write_line(f"{achieved:10.3e} <= {bar:7.0e}  {quantity:24s} {nodeid}")
