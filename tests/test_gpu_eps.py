"""GPU parity of the error-tolerant few-view solver (min psi(x) s.t.
||Ax - b|| <= eps, x >= 0, the extension the conclusions of Sec. 5 name)
against the oracle's ``fewview_eps_solve``.

* default step sizes: sigma = rho / lambda_max(K^T D(1) K), K = [A, -I], and
  the default tau, against the oracle's FP64 eigenvalue (1e-6);
* iterates on noisy few-view data with the ball constraint active
  (eps = the noise norm, and half of it) and inactive (eps > ||b||): x^k
  relative l2 1e-4, psi and ||Ax - b|| / ||b|| per iteration 1e-5 / 1e-4;
* eps = 0 is Algorithm 2 bit for bit at the same tau and sigma (with and
  without the per-iteration monitors);
* rejections: eps < 0 or not finite, sigma beyond the bound.
"""
import numpy as np
import pytest
import torch

from oracle import app as OA
from oracle import tv as OT
from paper_1609_06041_amd import ctpd
from paper_1609_06041_amd import synth as S

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def max_rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b) / np.abs(b)))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


def noisy_fewview(n, m, nb, seed):
    prob = S.make_problem(93, seed, n, m, nb, 8, 2e4, with_x_true=False)
    b = np.asarray(prob.b, np.float32).astype(np.float64)
    noise = float(np.linalg.norm(b - prob.b_true))
    return b, noise


def test_eps_default_steps_match_oracle(gpu, parity):
    n, m, nb = 48, 16, 70
    b, noise = noisy_fewview(n, m, nb, 0)
    st = OA.steps_fewview_eps(b, n)
    with ctpd.Operator(n, m, nb) as op:
        x, info = op.fewview_eps_solve(dev(b), noise, 3)
        x = host(x)
        assert info["norm_steps_a"] > 0
        parity("sigma", abs(info["sigma"] - st.sigma) / st.sigma, 1e-6)
        parity("tau", abs(info["tau"] - st.tau) / st.tau, 1e-6)
        parity("lambda_max(K^T D K)", abs(info["lambda_a"] - st.lambda_a) / st.lambda_a, 1e-6)
        # the second solve reuses the cached norm
        _, info2 = op.fewview_eps_solve(dev(b), noise, 1)
        assert info2["norm_steps_a"] == 0 and info2["sigma"] == info["sigma"]
    ref, _ = OA.fewview_eps_solve(b, n, noise, 3, tau=st.tau, sigma=st.sigma)
    parity("x", rel(x, ref.x), 1e-4)


@pytest.mark.parametrize("n,m,nb,frac,iters", [
    (48, 16, 70, 1.0, 30),     # eps = the noise norm
    (40, 12, 60, 0.5, 25),     # half of it
    (33, 9, 48, 0.0, 20),      # eps = 0 against the oracle too
])
def test_eps_solve_matches_oracle(gpu, parity, n, m, nb, frac, iters):
    b, noise = noisy_fewview(n, m, nb, 1)
    eps = frac * noise
    st = OA.steps_fewview_eps(b, n)

    def monitor(x, y, mu):
        return OT.tv_norm(x), OA.data_residual(x, b)

    ref, _ = OA.fewview_eps_solve(b, n, eps, iters, tau=st.tau, sigma=st.sigma, monitor=monitor)
    with ctpd.Operator(n, m, nb) as op:
        x, info = op.fewview_eps_solve(dev(b), eps, iters, tau=st.tau, sigma=st.sigma, record_cost=True,
                                       monitors=("resid",))
        x = host(x)
    psi_ref = [h[0] for h in ref.history]
    res_ref = [h[1] for h in ref.history]
    parity(f"x (eps = {frac:g} noise)", rel(x, ref.x), 1e-4)
    parity("psi history (max rel)", max_rel(info["cost"], psi_ref), 1e-5)
    parity("||Ax-b||/||b|| history (max rel)", max_rel(info["resid"], res_ref), 1e-4)


def test_eps_beyond_the_data_norm(gpu, parity):
    # x = 0 is feasible: the ball constraint never binds and the iterates lose their TV
    n, m, nb = 40, 12, 60
    b, _ = noisy_fewview(n, m, nb, 2)
    eps = 1.5 * float(np.linalg.norm(b))
    st = OA.steps_fewview_eps(b, n)
    ref, _ = OA.fewview_eps_solve(b, n, eps, 40, tau=st.tau, sigma=st.sigma)
    with ctpd.Operator(n, m, nb) as op:
        x, _ = op.fewview_eps_solve(dev(b), eps, 40, tau=st.tau, sigma=st.sigma)
        x = host(x)
    parity("x (eps > ||b||)", rel(x, ref.x), 1e-4)


@pytest.mark.parametrize("monitors", [(), ("resid",)])
def test_eps_zero_is_algorithm_2_bit_for_bit(gpu, monitors):
    n, m, nb = 64, 32, 96
    b, _ = noisy_fewview(n, m, nb, 3)
    st = OA.steps_fewview_eps(b, n)   # its sigma is within Algorithm 2's bound too
    with ctpd.Operator(n, m, nb) as op:
        kw = dict(tau=st.tau, sigma=st.sigma, record_cost=bool(monitors), monitors=monitors, return_state=True)
        xa, ia = op.fewview_solve(dev(b), 12, **kw)
        xa, mua = host(xa), host(ia["mu"])
        xe, ie = op.fewview_eps_solve(dev(b), 0.0, 12, **kw)
        xe, mue = host(xe), host(ie["mu"])
    np.testing.assert_array_equal(xe, xa)
    np.testing.assert_array_equal(mue, mua)
    if monitors:
        np.testing.assert_array_equal(ie["resid"], ia["resid"])
        np.testing.assert_array_equal(ie["cost"], ia["cost"])


def test_eps_rejections(gpu):
    n, m, nb = 32, 10, 48
    b, noise = noisy_fewview(n, m, nb, 4)
    st = OA.steps_fewview_eps(b, n)
    with ctpd.Operator(n, m, nb) as op:
        for bad in (-1.0, float("nan"), float("inf")):
            with pytest.raises(ctpd.CtpdError) as e:
                op.fewview_eps_solve(dev(b), bad, 2)
            assert e.value.code == ctpd.CTPD_EINVAL
        bound = 1.0 / (st.lambda_a * st.tau)   # 1 / lambda_max(K^T D(1) K)
        with pytest.raises(ctpd.CtpdError) as e:
            op.fewview_eps_solve(dev(b), noise, 2, tau=0.5, sigma=1.03 * bound)
        assert e.value.code == ctpd.CTPD_EINVAL
        _, info = op.fewview_eps_solve(dev(b), noise, 2, tau=0.5, sigma=0.97 * bound)
        assert info["sigma"] == 0.97 * bound


def test_eps_rmse_monitor_and_given_angles(gpu, parity):
    # a limited-angle scan (views over 120 degrees) and the Eq. 34 RMSE monitor
    n, m, nb = 40, 14, 60
    theta = np.linspace(0.0, 2.0 * np.pi / 3.0, m, endpoint=False)
    prob = S.make_problem(94, 0, n, m, nb, 8, None, with_x_true=True)
    x_true = np.asarray(prob.x_true, np.float64)
    from oracle import projector as OP
    b = np.asarray(OP.forward_project(x_true, m, nb, theta=theta), np.float32).astype(np.float64)
    eps = 0.01 * float(np.linalg.norm(b))
    # the oracle's error-tolerant solve takes uniform angles only: the
    # monitors are checked against the oracle's formulas (Eq. 34, Eq. 25's
    # residual) on the returned iterate
    with ctpd.Operator(n, m, nb, angles=theta) as op:
        x, info = op.fewview_eps_solve(dev(b), eps, 15, monitors=("rmse", "resid"), x_ref=dev(x_true))
        x = host(x)
    parity("rmse(x^K) vs the returned x", abs(info["rmse"][-1] - OA.rmse(x, x_true)) / OA.rmse(x, x_true), 1e-6)
    ref_res = float(np.linalg.norm(OP.forward_project(x, m, nb, theta=theta) - b) / np.linalg.norm(b))
    parity("||Ax-b||/||b|| vs the returned x", abs(info["resid"][-1] - ref_res) / ref_res, 1e-4)
