"""ctpd_project_noalloc (the projector that allocates nothing; its scratch is a
static device array) against ctpd_project, through the C ABI: two calls in a
row, the second on a smaller problem, so the second call runs on scratch the
first one left behind.  Bar: relative l2 1e-6 (both are Joseph's A in float32
with the same per-ray arithmetic; the no-allocation view table is computed on
the device instead of the host, which can move the last bits of the
geometry)."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1609_06041_amd import ctpd

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(torch.linalg.norm((a - b).double()) / torch.linalg.norm(b.double()))


def test_noalloc_projection_equals_project(gpu, parity):
    torch.manual_seed(0)
    for n, m, nb in [(200, 90, 290), (64, 45, 96)]:   # second call smaller
        x = torch.rand((n, n), dtype=torch.float32).cuda()
        with ctpd.Operator(n, m, nb) as op:
            ref = op.project(x)
            y = ctpd.project_noalloc(x, m, nb, stream=op.stream)
            torch.cuda.synchronize()
        parity(f"y {n}x{n} {m}x{nb}", rel(y, ref), 1e-6)


def test_noalloc_rejects_sizes_beyond_its_scratch(gpu):
    lib = ctpd.load()
    x = torch.zeros((8, 8), device="cuda")
    y = torch.zeros((8, 8), device="cuda")
    for n, m, nb in [(1025, 8, 8), (8, 4097, 8), (8, 8, 4097), (0, 8, 8)]:
        g = ctpd.Geometry(n, m, nb, 0, None)
        code = lib.ctpd_project_noalloc(ctypes.byref(g), None, ctypes.c_void_p(x.data_ptr()),
                                        ctypes.c_void_p(y.data_ptr()))
        assert code == ctpd.CTPD_EINVAL
    th = np.linspace(0.0, 3.0, 8)
    g, keep = ctpd._geometry(8, 8, 8, th)
    assert lib.ctpd_project_noalloc(ctypes.byref(g), None, ctypes.c_void_p(x.data_ptr()),
                                    ctypes.c_void_p(y.data_ptr())) == ctpd.CTPD_EINVAL
