"""GPU parity of the APP solvers (Algorithms 1, 1', 2) against the FP64 oracle.

The GPU runs in float32; the oracle in float64 on the same float32 inputs,
with the same tau and sigma.  Bars: iterate x^k relative l2 <= 1e-4, cost
(Eq. 1, or psi for few-view) relative <= 1e-5; operator norms from the
GPU's float64 Lanczos within 1e-6 of the oracle's eigenvalues.
"""
import math

import numpy as np
import pytest
import torch

from oracle import app as OA
from oracle import filters as OF
from oracle import projector as OP
from oracle import tv as OT
from paper_1609_06041_amd import ctpd
from paper_1609_06041_amd import synth as S

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def max_rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b) / np.abs(b)))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


def lowdose_inputs(n, m, nb, seed, n_ell=8, i0=1e4):
    prob = S.make_problem(90, seed, n, m, nb, n_ell, i0, with_x_true=False)
    b32, w32 = S.as_f32_inputs(prob)
    return b32.astype(np.float64), w32.astype(np.float64)


@pytest.mark.parametrize("n,m,nb,beta,iters", [(64, 90, 96, 0.01, 50), (45, 30, 70, 0.02, 20),
                                               (64, 90, 96, 0.0, 20), (33, 17, 49, 0.05, 5)])
def test_lowdose_solve_matches_oracle(gpu, parity, n, m, nb, beta, iters):
    b, w = lowdose_inputs(n, m, nb, seed=n + m)
    st = OA.steps_lowdose(w, n)
    ref, _ = OA.lowdose_solve(b, w, beta, n, iters, tau=st.tau, sigma=st.sigma, record_cost=True)
    with ctpd.Operator(n, m, nb) as op:
        x, info = op.lowdose_solve(dev(b), dev(w), beta, iters, tau=st.tau, sigma=st.sigma, record_cost=True,
                                   return_state=True)
        x = host(x)
        mu = host(info["mu"])
    parity("x", rel(x, ref.x), 1e-4)
    parity("mu", rel(mu, ref.mu), 1e-4)
    f_gpu = OA.cost_lowdose(x, b, w, beta)
    f_ref = OA.cost_lowdose(ref.x, b, w, beta)
    parity("cost", abs(f_gpu - f_ref) / f_ref, 1e-5)
    # per-iteration cost reported by the GPU (float64 sums of float32 residuals):
    # the early iterates' residual Ax - b cancels to ~1e-2 of b, which lifts
    # float32 rounding to ~1e-5 of f there
    parity("cost history (max rel)", max_rel(info["cost"], ref.history), 3e-5)
    assert x.min() >= 0.0


def test_lowdose_default_steps_match_oracle(gpu, parity):
    n, m, nb = 64, 90, 96
    b, w = lowdose_inputs(n, m, nb, seed=0)
    st = OA.steps_lowdose(w, n)
    with ctpd.Operator(n, m, nb) as op:
        x, info = op.lowdose_solve(dev(b), dev(w), 0.01, 10)
        x = host(x)
    assert info["kappa"] == pytest.approx(st.kappa, rel=1e-12)
    assert info["tau"] == pytest.approx(st.tau, rel=1e-12)
    assert info["lambda_a"] == pytest.approx(st.lambda_a, rel=1e-6)
    assert info["lambda_h"] == pytest.approx(st.lambda_h, rel=1e-6)
    assert info["sigma"] == pytest.approx(st.sigma, rel=1e-6)
    ref, _ = OA.lowdose_solve(b, w, 0.01, n, 10, tau=st.tau, sigma=st.sigma)
    parity("x", rel(x, ref.x), 1e-4)


def test_second_solve_reuses_the_geometry_norm(gpu, parity):
    # with the default tau, kappa * lambda_max(A^T D A) depends on the geometry only
    n, m, nb = 64, 90, 96
    b1, w1 = lowdose_inputs(n, m, nb, seed=11)
    b2, w2 = lowdose_inputs(n, m, nb, seed=12, i0=3e4)
    st2 = OA.steps_lowdose(w2, n)
    with ctpd.Operator(n, m, nb) as op:
        _, i1 = op.lowdose_solve(dev(b1), dev(w1), 0.01, 2)
        x, i2 = op.lowdose_solve(dev(b2), dev(w2), 0.01, 10)
        x = host(x)
    assert i1["norm_steps_a"] > 0 and i2["norm_steps_a"] == 0
    assert i2["lambda_a"] == pytest.approx(st2.lambda_a, rel=1e-6)
    assert i2["lambda_h"] == pytest.approx(st2.lambda_h, rel=1e-6)
    assert i2["sigma"] == pytest.approx(st2.sigma, rel=1e-6)
    ref, _ = OA.lowdose_solve(b2, w2, 0.01, n, 10, tau=st2.tau, sigma=st2.sigma)
    parity("x", rel(x, ref.x), 1e-4)


@pytest.mark.parametrize("n,m,nb,iters", [(64, 32, 96, 20), (50, 12, 75, 10)])
def test_fewview_solve_matches_oracle(gpu, parity, n, m, nb, iters):
    prob = S.make_problem(91, n, n, m, nb, 8, None, with_x_true=False)
    b = np.asarray(prob.b, np.float32).astype(np.float64)
    st = OA.steps_fewview(b, n)
    ref, _ = OA.fewview_solve(b, n, iters, tau=st.tau, sigma=st.sigma, record_cost=True)
    with ctpd.Operator(n, m, nb) as op:
        x, info = op.fewview_solve(dev(b), iters, tau=st.tau, sigma=st.sigma, record_cost=True)
        x = host(x)
    parity("x", rel(x, ref.x), 1e-4)
    parity("psi", abs(OT.tv_norm(x) - OT.tv_norm(ref.x)) / OT.tv_norm(ref.x), 1e-5)
    parity("cost history (max rel)", max_rel(info["cost"], ref.history), 1e-5)


def test_fewview_default_steps_match_oracle(gpu, parity):
    n, m, nb = 64, 32, 96
    prob = S.make_problem(92, 0, n, m, nb, 8, None, with_x_true=False)
    b = np.asarray(prob.b, np.float32).astype(np.float64)
    st = OA.steps_fewview(b, n)
    with ctpd.Operator(n, m, nb) as op:
        x, info = op.fewview_solve(dev(b), 3)
        x = host(x)
    assert info["sigma"] == pytest.approx(st.sigma, rel=1e-6)
    assert info["tau"] == pytest.approx(st.tau, rel=1e-6)
    ref, _ = OA.fewview_solve(b, n, 3, tau=st.tau, sigma=st.sigma)
    parity("x", rel(x, ref.x), 1e-4)


def test_first_iteration_full_size(gpu, parity):
    # one Algorithm-1 iteration on the 512^2 / 720 x 736 workload, whole image
    n, m, nb = 512, 720, 736
    prob, spec = S.workload_problem("lowdose_512", with_x_true=False)
    b32, w32 = S.as_f32_inputs(prob)
    b, w = b32.astype(np.float64), w32.astype(np.float64)
    kappa = float((1.0 / w).mean())
    tau = OA.default_tau_lowdose(kappa, m)
    # fixed, so the oracle does not need the full-size eigenvalues; below the
    # Eq. 16 bound (about 0.87 here), which the library checks
    sigma = 0.8
    ref, _ = OA.lowdose_solve(b, w, spec["beta"], n, 1, tau=tau, sigma=sigma)
    with ctpd.Operator(n, m, nb) as op:
        x, info = op.lowdose_solve(dev(b), dev(w), spec["beta"], 1, tau=tau, sigma=sigma, return_state=True)
        x, mu = host(x), host(info["mu"])
    parity("x", rel(x, ref.x), 1e-4)
    parity("mu", rel(mu, ref.mu), 1e-4)


def test_zero_iterations_return_zero_image(gpu):
    n, m, nb = 16, 8, 24
    b, w = lowdose_inputs(n, m, nb, seed=3)
    with ctpd.Operator(n, m, nb) as op:
        x, info = op.lowdose_solve(dev(b), dev(w), 0.1, 0, tau=0.1, sigma=0.1)
        assert host(x).max() == 0.0 and info["iters_done"] == 0


def test_invalid_weights_and_data_are_rejected(gpu):
    n, m, nb = 16, 8, 24
    b, w = lowdose_inputs(n, m, nb, seed=4)
    w_bad = w.copy()
    w_bad[3, 5] = 0.0
    b_bad = b.copy()
    b_bad[1, 1] = np.nan
    with ctpd.Operator(n, m, nb) as op:
        with pytest.raises(ctpd.CtpdError) as e:
            op.lowdose_solve(dev(b), dev(w_bad), 0.1, 3)
        assert e.value.code == ctpd.CTPD_EDOMAIN
        with pytest.raises(ctpd.CtpdError) as e:
            op.lowdose_solve(dev(b_bad), dev(w), 0.1, 3)
        assert e.value.code == ctpd.CTPD_EDOMAIN
        with pytest.raises(ctpd.CtpdError) as e:
            op.fewview_solve(dev(b_bad), 3)
        assert e.value.code == ctpd.CTPD_EDOMAIN
        with pytest.raises(ctpd.CtpdError) as e:
            op.lowdose_solve(dev(b), dev(w), -1.0, 3)
        assert e.value.code == ctpd.CTPD_EINVAL
        with pytest.raises(ctpd.CtpdError) as e:
            op.lowdose_solve(dev(b), dev(w), 0.1, 3, norm_steps=513)
        assert e.value.code == ctpd.CTPD_EINVAL


@pytest.mark.parametrize("n,m,nb", [(128, 180, 184), (48, 10, 1100)])
def test_lambda_h_equals_the_largest_per_view_eigenvalue(gpu, n, m, nb):
    # W^-1/2 D W^-1/2 is block diagonal over views: lambda_h is the largest
    # eigenvalue of the m dense nb x nb blocks (brute force here).  The GPU
    # stops the chains of views whose bound (symbol maximum x max 1/w) falls
    # below the best Ritz value, which must not change the result.  Up to 1024
    # bins a round of a chain is one launch; 1100 bins take the per-step path
    # (batched FP64 MFMA filter, then the recurrence kernel).
    from scipy.linalg import eigh, toeplitz
    from oracle.filters import smoothed_ramp_taps
    b, w = lowdose_inputs(n, m, nb, seed=21, n_ell=12, i0=2e4)
    with ctpd.Operator(n, m, nb) as op:
        _, info = op.lowdose_solve(dev(b), dev(w), 0.01, 1)
    h = smoothed_ramp_taps(nb, m, info["tau"], info["kappa"])
    T = toeplitz(h[nb - 1:])
    rs = np.sqrt(1.0 / w)
    lam = max(eigh(rs[v][:, None] * T * rs[v][None, :], eigvals_only=True, subset_by_index=[nb - 1, nb - 1])[0]
              for v in range(m))
    assert info["lambda_h"] == pytest.approx(lam, rel=1e-6)


@pytest.mark.parametrize("algo", ["lowdose", "fewview"])
def test_fused_filter_inputs_equal_the_prologue_path(gpu, algo):
    # without the cost monitor the projector writes the dual-update residual
    # and the dual update writes the next extrapolation's input; with it, the
    # filters form them in their prologues -- the same arithmetic, so the
    # iterates agree bit for bit
    n, m, nb = 64, 90, 96
    b, w = lowdose_inputs(n, m, nb, seed=31)
    with ctpd.Operator(n, m, nb) as op:
        if algo == "lowdose":
            x0, i0 = op.lowdose_solve(dev(b), dev(w), 0.01, 12)
            x1, i1 = op.lowdose_solve(dev(b), dev(w), 0.01, 12, record_cost=True)
        else:
            x0, i0 = op.fewview_solve(dev(b), 12)
            x1, i1 = op.fewview_solve(dev(b), 12, record_cost=True)
        assert i0["sigma"] == i1["sigma"] and i0["tau"] == i1["tau"]
        np.testing.assert_array_equal(host(x0), host(x1))


def test_lowdose_with_given_angles_matches_oracle(gpu, parity):
    # limited-angle scan (135 degrees, irregular spacing): default step sizes
    # from the GPU's Lanczos chains on that geometry, then 10 iterations
    n, m, nb = 48, 30, 70
    th = np.sort(np.random.default_rng(31).uniform(0.1, 0.1 + 0.75 * np.pi, m))
    b, w = lowdose_inputs(n, m, nb, seed=31)
    st = OA.steps_lowdose(w, n, theta=th)
    ref, _ = OA.lowdose_solve(b, w, 0.02, n, 10, tau=st.tau, sigma=st.sigma, theta=th)
    with ctpd.Operator(n, m, nb, angles=th) as op:
        x, info = op.lowdose_solve(dev(b), dev(w), 0.02, 10)
        x = host(x)
    assert info["tau"] == pytest.approx(st.tau, rel=1e-12)
    assert info["lambda_a"] == pytest.approx(st.lambda_a, rel=1e-6)
    assert info["sigma"] == pytest.approx(st.sigma, rel=1e-6)
    parity("x", rel(x, ref.x), 1e-4)


def test_lowdose_tv_term_is_pinned(gpu, parity):
    # A TV weight large enough that the prox coupling moves the iterates:
    # the oracle's beta > 0 and beta = 0 trajectories differ by more than 100x
    # the 1e-4 parity bar, so a GPU solve with the TV term dropped or
    # mis-weighted (lambda = tau beta, Algorithm 1 Step 2) fails this test.
    n, m, nb, beta, iters = 64, 90, 96, 100.0, 50
    b, w = lowdose_inputs(n, m, nb, seed=n + m)
    st = OA.steps_lowdose(w, n)
    ref, _ = OA.lowdose_solve(b, w, beta, n, iters, tau=st.tau, sigma=st.sigma, record_cost=True)
    ref0, _ = OA.lowdose_solve(b, w, 0.0, n, iters, tau=st.tau, sigma=st.sigma)
    gap = rel(ref.x, ref0.x)
    print(f"oracle x^{iters}: beta = {beta} vs beta = 0 differ by {gap:.3e} relative")
    assert gap >= 100 * 1e-4
    with ctpd.Operator(n, m, nb) as op:
        x, info = op.lowdose_solve(dev(b), dev(w), beta, iters, record_cost=True)
        x = host(x)
    parity("x", rel(x, ref.x), 1e-4)
    parity("cost history (max rel)", max_rel(info["cost"], ref.history), 3e-5)
    parity("psi", abs(OT.tv_norm(x) - OT.tv_norm(ref.x)) / OT.tv_norm(ref.x), 1e-4)


# ---- step sizes given by the caller are checked (Eq. 16; Algorithms 1 and 2) ----

def test_lowdose_sigma_beyond_the_bound_is_rejected(gpu):
    n, m, nb = 48, 30, 70
    b, w = lowdose_inputs(n, m, nb, seed=41)
    st = OA.steps_lowdose(w, n)
    bound = min(2.0 / st.lambda_h, 1.0 / (st.tau * st.lambda_a))
    with ctpd.Operator(n, m, nb) as op:
        for sig in (1.02 * bound, 3.0 * bound):
            with pytest.raises(ctpd.CtpdError) as e:
                op.lowdose_solve(dev(b), dev(w), 0.01, 3, tau=st.tau, sigma=sig)
            assert e.value.code == ctpd.CTPD_EINVAL
            assert "sigma" in str(e.value)
        # just inside the bound it runs, and the report carries the norms it was checked with
        x, info = op.lowdose_solve(dev(b), dev(w), 0.01, 3, tau=st.tau, sigma=0.98 * bound)
        assert info["sigma"] == 0.98 * bound
        assert info["lambda_a"] == pytest.approx(st.lambda_a, rel=1e-6)
        assert info["lambda_h"] == pytest.approx(st.lambda_h, rel=1e-6)
        # a tau other than the default: lambda_A at that tau (D depends on tau)
        tau2 = 3.0 * st.tau
        st2 = OA.steps_lowdose(w, n, tau=tau2)
        bound2 = min(2.0 / st2.lambda_h, 1.0 / (tau2 * st2.lambda_a))
        with pytest.raises(ctpd.CtpdError) as e:
            op.lowdose_solve(dev(b), dev(w), 0.01, 3, tau=tau2, sigma=1.05 * bound2)
        assert e.value.code == ctpd.CTPD_EINVAL
        _, info2 = op.lowdose_solve(dev(b), dev(w), 0.01, 3, tau=tau2, sigma=0.9 * bound2)
        assert info2["lambda_a"] == pytest.approx(st2.lambda_a, rel=1e-6)


def test_fewview_sigma_beyond_the_bound_is_rejected(gpu):
    n, m, nb = 48, 16, 70
    prob = S.make_problem(92, 7, n, m, nb, 8, None, with_x_true=False)
    b = np.asarray(prob.b, np.float32).astype(np.float64)
    st = OA.steps_fewview(b, n)
    bound = 1.0 / (st.lambda_a * st.tau)   # 1 / lambda_max(A^T D(1) A)
    with ctpd.Operator(n, m, nb) as op:
        with pytest.raises(ctpd.CtpdError) as e:
            op.fewview_solve(dev(b), 3, tau=0.5, sigma=1.03 * bound)
        assert e.value.code == ctpd.CTPD_EINVAL
        _, info = op.fewview_solve(dev(b), 3, tau=0.5, sigma=0.97 * bound)
        assert info["sigma"] == 0.97 * bound


def test_comparator_steps_beyond_their_bounds_are_rejected(gpu):
    from oracle import comparators as OC
    n, m, nb = 40, 24, 57
    b, w = lowdose_inputs(n, m, nb, seed=43)
    with ctpd.Operator(n, m, nb) as op:
        # D = I ablation: sigma < min(2/lambda_h, 1/(tau lambda_A))
        sti = OA.steps_lowdose_identity(w, n)
        bi = min(2.0 / sti.lambda_h, 1.0 / (sti.tau * sti.lambda_a))
        with pytest.raises(ctpd.CtpdError) as e:
            op.app_identity_lowdose_solve(dev(b), dev(w), 0.01, 2, tau=sti.tau, sigma=1.05 * bi)
        assert e.value.code == ctpd.CTPD_EINVAL
        # GIST: gamma < 2 / lambda_max(A^T W A)
        stg = OC.gist_steps(w, n)
        with pytest.raises(ctpd.CtpdError) as e:
            op.gist_lowdose_solve(dev(b), dev(w), 0.01, 2, gamma=1.05 * 2.0 / stg.norm)
        assert e.value.code == ctpd.CTPD_EINVAL
        op.gist_lowdose_solve(dev(b), dev(w), 0.01, 2, gamma=0.9 * 2.0 / stg.norm)
        # Chambolle-Pock: s t (lambda_max(A^T A) + 8) < 1
        stc = OC.cp_steps(n, m, nb)
        big = 1.05 / np.sqrt(stc.norm + 8.0)
        with pytest.raises(ctpd.CtpdError) as e:
            op.cp_fewview_solve(dev(b), 2, t=big, s=big)
        assert e.value.code == ctpd.CTPD_EINVAL
