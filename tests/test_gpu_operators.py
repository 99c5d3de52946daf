"""GPU parity of the single operators against the FP64 oracle, through the C ABI.

A, A^T, D: relative l2 error <= 1e-5 (float32 kernels vs float64 oracle on the
same float32 inputs); filter taps to 1e-12 of h[0]; the TV prox (x and the
dual field) to 1e-5.  Sizes span several tiles with ragged tails, the 45 and
135 degree ties, the degenerate 1-pixel case, and the full 512 x 720 x 736
workload.
"""
import math

import numpy as np
import pytest
import torch

from oracle import filters as OF
from oracle import projector as OP
from oracle import tv as OT
from paper_1609_06041_amd import ctpd
from paper_1609_06041_amd import synth as S

pytestmark = pytest.mark.gpu

TOL = 1e-5


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


GEOMS = [(1, 1, 1), (7, 5, 11), (64, 90, 96), (100, 36, 143), (129, 33, 200), (64, 32, 96), (384, 720, 546)]


@pytest.mark.parametrize("n,m,nb", GEOMS)
def test_project_matches_oracle(gpu, parity, n, m, nb):
    rng = np.random.default_rng(n + 7 * m + 13 * nb)
    x = f32(rng.random((n, n)))
    with ctpd.Operator(n, m, nb) as op:
        y = host(op.project(dev(x)))
    ref = OP.forward_project(x, m, nb)
    parity("y", rel(y, ref), TOL)


@pytest.mark.parametrize("n,m,nb", GEOMS)
def test_backproject_matches_oracle(gpu, parity, n, m, nb):
    rng = np.random.default_rng(3 * n + m + nb)
    y = f32(rng.standard_normal((m, nb)))
    with ctpd.Operator(n, m, nb) as op:
        x = host(op.backproject(dev(y)))
    ref = OP.back_project(y, n)
    parity("x", rel(x, ref), TOL)


def test_gpu_adjoint_identity(gpu):
    n, m, nb = 200, 90, 290
    rng = np.random.default_rng(5)
    x = f32(rng.random((n, n)))
    y = f32(rng.standard_normal((m, nb)))
    with ctpd.Operator(n, m, nb) as op:
        ax = host(op.project(dev(x)))
        aty = host(op.backproject(dev(y)))
    lhs, rhs = float((ax * y).sum()), float((x * aty).sum())
    assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(ax) * np.linalg.norm(y)


def test_phantom_projection_and_backprojection_full_size(gpu, parity):
    # the 512^2 image, 720 views x 736 bins workload, whole outputs
    n, m, nb = 512, 720, 736
    prob = S.make_problem(1, 0, n, m, nb, 20, None, with_x_true=True)
    x = f32(prob.x_true)
    b = f32(prob.b)
    with ctpd.Operator(n, m, nb) as op:
        y = host(op.project(dev(x)))
        xb = host(op.backproject(dev(b)))
    parity("y", rel(y, OP.forward_project(x, m, nb)), TOL)
    parity("xb", rel(xb, OP.back_project(b, n)), TOL)


@pytest.mark.parametrize("m,nb,tau,kappa", [(90, 96, 1.0, 0.0), (90, 96, 2.8e-6, 1.6e-4), (720, 736, 0.01, 0.0),
                                            (720, 736, 3.4e-6, 1.5e-5), (5, 37, 0.3, 0.02), (33, 1, 1.0, 0.5)])
def test_filter_taps_match_oracle(gpu, m, nb, tau, kappa):
    with ctpd.Operator(16, m, nb) as op:
        taps = op.filter_taps(tau, kappa)
    ref = OF.smoothed_ramp_taps(nb, m, tau, kappa)
    assert np.abs(taps - ref).max() <= 1e-12 * abs(ref[nb - 1])


@pytest.mark.parametrize("m,nb,kappa", [(90, 96, 0.0), (90, 96, 1.6e-4), (720, 736, 0.0), (720, 736, 1.5e-5),
                                        (32, 736, 0.0), (5, 37, 0.02), (33, 65, 0.0), (1, 1, 0.1), (47, 130, 0.3),
                                        (90, 546, 1.6e-4), (17, 3, 0.05)])
def test_ramp_filter_matches_oracle(gpu, parity, m, nb, kappa):
    rng = np.random.default_rng(m * nb)
    s = f32(rng.standard_normal((m, nb)))
    tau = 0.7 if kappa == 0.0 else math.pi * kappa / (2 * m)
    with ctpd.Operator(8, m, nb) as op:
        out = host(op.ramp_filter(dev(s), tau, kappa))
    ref = OF.apply_filter(s, OF.smoothed_ramp_taps(nb, m, tau, kappa))
    parity("out", rel(out, ref), TOL)


@pytest.mark.parametrize("m,nb", [(17, 1024), (5, 1056), (3, ctpd.MAX_BINS)])
def test_ramp_filter_long_rows_match_oracle(gpu, parity, m, nb):
    # 1024 bins: the longest row of the unrolled step form (8 steps of 32 bins
    # per wave); 1056: the first of the looped form; the maximum row length
    rng = np.random.default_rng(nb + m)
    s = f32(rng.standard_normal((m, nb)))
    tau, kappa = math.pi * 2e-4 / (2 * m), 2e-4
    with ctpd.Operator(8, m, nb) as op:
        out = host(op.ramp_filter(dev(s), tau, kappa))
    ref = OF.apply_filter(s, OF.smoothed_ramp_taps(nb, m, tau, kappa))
    parity("out", rel(out, ref), TOL)


@pytest.mark.parametrize("m,nb", [(90, 546), (40, 96), (21, 70), (33, 65), (7, 1056)])
def test_ramp_filter_load_widths_agree(gpu, m, nb):
    # the filter reads its input 16, 8 or 4 bytes a lane, as the row length
    # and the input's address allow; every width must give the same bits
    rng = np.random.default_rng(5 * m + nb)
    s = f32(rng.standard_normal((m, nb)))
    tau, kappa = math.pi * 1e-4 / (2 * m), 1e-4
    with ctpd.Operator(8, m, nb) as op:
        aligned = host(op.ramp_filter(dev(s), tau, kappa))
        buf = torch.zeros(m * nb + 4, device="cuda")
        for off in (1, 2, 3):
            view = buf[off:off + m * nb].view(m, nb)
            view.copy_(dev(s))
            np.testing.assert_array_equal(host(op.ramp_filter(view, tau, kappa)), aligned)


@pytest.mark.parametrize("m,nb,kappa", [(90, 96, 1.6e-4), (720, 736, 0.0), (5, 37, 0.02), (33, 65, 0.0),
                                        (1, 1, 0.1), (47, 130, 0.3)])
def test_ramp_filter_f64_matches_oracle(gpu, parity, m, nb, kappa):
    rng = np.random.default_rng(m * nb + 1)
    s = rng.standard_normal((m, nb))
    tau = 0.7 if kappa == 0.0 else math.pi * kappa / (2 * m)
    with ctpd.Operator(8, m, nb) as op:
        out = op.ramp_filter_f64(torch.from_numpy(s).cuda(), tau, kappa)
        torch.cuda.synchronize()
        out = out.cpu().numpy()
    ref = OF.apply_filter(s, OF.smoothed_ramp_taps(nb, m, tau, kappa))
    parity("out", rel(out, ref), 1e-12)


def test_ramp_filter_on_phantom_sinogram(gpu, parity):
    n, m, nb = 512, 720, 736
    prob = S.make_problem(1, 0, n, m, nb, 20, 5e4, with_x_true=False)
    b = f32(prob.b)
    kappa = float((1.0 / f32(prob.w)).mean())
    tau = math.pi * kappa / (2 * m)
    with ctpd.Operator(n, m, nb) as op:
        out = host(op.ramp_filter(dev(b), tau, kappa))
    ref = OF.apply_filter(b, OF.smoothed_ramp_taps(nb, m, tau, kappa))
    parity("out", rel(out, ref), TOL)


def _unit_ball_field(rng, n):
    p = rng.standard_normal((2, n, n))
    p /= np.maximum(1.0, np.hypot(p[0], p[1]))[None]
    return f32(p)


@pytest.mark.parametrize("n,lam,n_iter", [(7, 0.05, 1), (64, 0.05, 10), (129, 2e-3, 10), (64, 0.0, 10),
                                          (100, 0.3, 25), (1, 0.1, 3)])
def test_tv_prox_matches_oracle(gpu, parity, n, lam, n_iter):
    rng = np.random.default_rng(n + n_iter)
    z = np.zeros((n, n))
    z[n // 4:3 * n // 4, n // 3:2 * n // 3] = 1.0
    z = f32(z + 0.2 * rng.standard_normal((n, n)))
    p0 = _unit_ball_field(rng, n)
    with ctpd.Operator(n, 4, 8) as op:
        pd = dev(p0)
        x, pd = op.tv_prox(dev(z), lam, pd, n_iter=n_iter)
        x, p = host(x), host(pd)
    xr, p1, p2 = OT.tv_prox(z, lam, p0[0].copy(), p0[1].copy(), n_iter)
    parity("x", rel(x, xr), TOL)
    parity("p", rel(p, np.stack([p1, p2])), TOL)
    assert x.min() >= 0.0


# ---- given view angles --------------------------------------------------

ANGLE_SETS = {
    # limited angle (120 degrees), irregular, with both diagonals and angles past pi and below 0
    "limited": (96, 50, 140, np.linspace(0.2, 0.2 + 2 * np.pi / 3, 50)),
    "irregular": (70, 37, 101, np.sort(np.random.default_rng(11).uniform(-1.0, 4.5, 37))),
    "diagonals": (33, 6, 48, np.array([np.pi / 4, 3 * np.pi / 4, -np.pi / 4, 5 * np.pi / 4, 0.0, np.pi / 2])),
}


@pytest.mark.parametrize("name", sorted(ANGLE_SETS))
def test_project_and_backproject_with_given_angles_match_oracle(gpu, parity, name):
    n, m, nb, th = ANGLE_SETS[name]
    rng = np.random.default_rng(m)
    x = f32(rng.random((n, n)))
    yb = f32(rng.standard_normal((m, nb)))
    with ctpd.Operator(n, m, nb, angles=th) as op:
        y = host(op.project(dev(x)))
        xb = host(op.backproject(dev(yb)))
    parity("y", rel(y, OP.forward_project(x, m, nb, theta=th)), TOL)
    parity("xb", rel(xb, OP.back_project(yb, n, theta=th)), TOL)


def test_uniform_angles_given_equal_the_default_scan(gpu):
    # the default scan spelled out (m = 90 has no 45-degree view index tie
    # at 4v = m): the same view tables, so the same results bit for bit
    n, m, nb = 64, 90, 96
    th = np.arange(m) * np.pi / m
    rng = np.random.default_rng(12)
    x, yb = dev(rng.random((n, n))), dev(rng.standard_normal((m, nb)))
    with ctpd.Operator(n, m, nb) as a, ctpd.Operator(n, m, nb, angles=th) as b:
        assert torch.equal(a.project(x), b.project(x))
        assert torch.equal(a.backproject(yb), b.backproject(yb))
