"""GPU convergence monitors against the FP64 oracle, per iteration.

The solvers' report carries, for every iteration k, float64 sums over the
iterate (x^k, mu^k) computed on the device:

* the partial primal-dual gap f(x) - L(x, mu) = 1/2 ||W^1/2 (Ax - b) - W^-1/2 mu||^2
  (Eq. 10 with the change of variables and the theorem after it);
* the data residual ||Ax - b|| / ||b|| (the constraint of Eq. 25);
* the RMSE against a reference image (Eq. 34).

Bars: RMSE 1e-5 relative (a sum of squares of x - x_ref, which does not cancel);
residual 1e-4 (A x nearly cancels b, so the iterate's ~1e-6 relative float32
error is amplified by |Ax| / |Ax - b|); gap 1e-3 (W^1/2 (Ax - b) and
W^-1/2 mu cancel further as the iteration converges, and each carries the
float32 error of x and mu times w ~ 1e4).
"""
import numpy as np
import pytest
import torch

from oracle import app as OA
from oracle import filters as OF
from paper_1609_06041_amd import ctpd
from paper_1609_06041_amd import synth as S

pytestmark = pytest.mark.gpu


def max_rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b) / np.abs(b)))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


@pytest.mark.parametrize("n,m,nb,beta,iters", [(64, 90, 96, 0.01, 20), (45, 30, 70, 2.0, 15)])
def test_lowdose_monitors_match_oracle(gpu, parity, n, m, nb, beta, iters):
    prob = S.make_problem(96, n, n, m, nb, 8, 1e4, with_x_true=True)
    b32, w32 = S.as_f32_inputs(prob)
    b, w, xt = b32.astype(np.float64), w32.astype(np.float64), f32(prob.x_true)
    st = OA.steps_lowdose(w, n)
    h = OF.smoothed_ramp_taps(nb, m, st.tau, st.kappa)
    mon = lambda x, mu: (OA.partial_gap(x, mu, b, w), OA.data_residual(x, b), OA.rmse(x, xt))
    ref = OA.app_solve(b, n, iters, st.tau, st.sigma, h, beta=beta, winv=1.0 / w, monitor=mon)
    gap, res, rm = (np.array(v) for v in zip(*ref.history))
    with ctpd.Operator(n, m, nb) as op:
        _, info = op.lowdose_solve(dev(b), dev(w), beta, iters, tau=st.tau, sigma=st.sigma,
                                   monitors=("gap", "resid", "rmse"), x_ref=dev(xt))
    parity("gap history (max rel)", max_rel(info["gap"], gap), 1e-3)
    parity("resid history (max rel)", max_rel(info["resid"], res), 1e-4)
    parity("rmse history (max rel)", max_rel(info["rmse"], rm), 1e-5)
    assert np.all(info["gap"] >= 0.0)


def test_fewview_monitors_match_oracle(gpu, parity):
    n, m, nb, iters = 64, 32, 96, 20
    prob = S.make_problem(97, 0, n, m, nb, 8, None, with_x_true=True)
    b, xt = f32(prob.b), f32(prob.x_true)
    st = OA.steps_fewview(b, n)
    mon = lambda x, mu: (OA.data_residual(x, b), OA.rmse(x, xt))
    ref = OA.app_solve(b, n, iters, st.tau, st.sigma, OF.ramp_taps(nb, m, st.tau), beta=1.0, winv=None,
                       monitor=mon)
    res, rm = (np.array(v) for v in zip(*ref.history))
    with ctpd.Operator(n, m, nb) as op:
        _, info = op.fewview_solve(dev(b), iters, tau=st.tau, sigma=st.sigma, monitors=("resid", "rmse"),
                                   x_ref=dev(xt))
        with pytest.raises(ctpd.CtpdError) as e:   # the partial gap is a low-dose quantity
            op.fewview_solve(dev(b), 2, monitors=("gap",))
        assert e.value.code == ctpd.CTPD_EINVAL
        with pytest.raises(ctpd.CtpdError) as e:   # rmse needs the reference image
            op.fewview_solve(dev(b), 2, monitors=("rmse",))
        assert e.value.code == ctpd.CTPD_EINVAL
    parity("resid history (max rel)", max_rel(info["resid"], res), 1e-4)
    parity("rmse history (max rel)", max_rel(info["rmse"], rm), 1e-5)


def test_monitors_leave_the_iterates_unchanged(gpu):
    # asking for monitors switches the solver to the filters' prologue path,
    # whose arithmetic is the fused path's: the iterates agree bit for bit
    n, m, nb = 48, 30, 70
    prob = S.make_problem(98, 0, n, m, nb, 8, 1e4, with_x_true=True)
    b32, w32 = S.as_f32_inputs(prob)
    with ctpd.Operator(n, m, nb) as op:
        x0, _ = op.lowdose_solve(dev(b32), dev(w32), 0.05, 8)
        x1, _ = op.lowdose_solve(dev(b32), dev(w32), 0.05, 8, monitors=("gap", "resid", "rmse"),
                                 x_ref=dev(prob.x_true))
        assert torch.equal(x0, x1)
