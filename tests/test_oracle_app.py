"""Pins for the APP solvers (Algorithms 1, 1', 2), step sizes and monitors.

* Algorithm 1' (beta = 0) must converge to the exact WLS minimiser with
  x >= 0, computed independently by NNLS on the dense system.
* Algorithm 1 must reach the same optimum as an independent Chambolle-Pock
  solve of Eq. 1 written here from its published definition.
* At the optimum the partial gap f(x) - L(x, mu) (Eqs. 10 and the duality
  theorem) vanishes.
* Algorithm 2 on consistent noiseless data drives Ax - b to zero with
  psi(x) no larger than psi(x_true).
* The simplified extrapolation of Eqs. 18 / 29 equals its defining form.
* The largest-eigenvalue routine equals a dense eigendecomposition.
"""
import math

import numpy as np
import pytest
from scipy.optimize import nnls

from oracle import app as AP
from oracle import filters as F
from oracle import projector as P
from oracle import tv as T


def _small_problem(seed, n=8, m=12, nb=12, noise=0.05):
    rng = np.random.default_rng(seed)
    xt = np.zeros((n, n))
    xt[2:6, 3:7] = 1.0
    xt[4:7, 1:3] = 0.5
    b = P.forward_project(xt, m, nb) + noise * rng.standard_normal((m, nb))
    w = rng.uniform(0.5, 2.0, (m, nb))
    return xt, b, w


def test_wls_solve_converges_to_nnls():
    n, m, nb = 8, 12, 12
    _, b, w = _small_problem(5, n, m, nb)
    a = P.dense_matrix(n, m, nb)
    sw = np.sqrt(w).ravel()
    ref, _ = nnls(sw[:, None] * a, sw * b.ravel())
    kappa = float((1.0 / w).mean())
    res, st = AP.lowdose_solve(b, w, 0.0, n, 1500, tau=3 * np.pi * kappa / (2.0 * m))
    assert st.sigma > 0 and st.tau > 0
    np.testing.assert_allclose(res.x.ravel(), ref, atol=1e-9)


def _chambolle_pock_tv_wls(a, b, w, beta, n, iters):
    # Chambolle & Pock (2011), Algorithm 1 with K = [A; grad], F1*(y) =
    # 1/2 ||y||^2_{W^-1} + <y, b>, F2* = indicator of {|q_j| <= beta},
    # G = indicator of x >= 0, and primal extrapolation theta = 1.
    lk = math.sqrt(np.linalg.norm(a, 2) ** 2 + 8.0)
    s = t = 0.99 / lk
    x = np.zeros(n * n)
    xb = x.copy()
    y = np.zeros(a.shape[0])
    q1 = np.zeros((n, n))
    q2 = np.zeros((n, n))
    for _ in range(iters):
        y = (y + s * (a @ xb - b)) / (1.0 + s / w)
        g1, g2 = T.grad(xb.reshape(n, n))
        q1, q2 = q1 + s * g1, q2 + s * g2
        sc = np.maximum(1.0, np.hypot(q1, q2) / beta)
        q1, q2 = q1 / sc, q2 / sc
        xo = x
        x = np.maximum(0.0, x - t * (a.T @ y - T.div(q1, q2).ravel()))
        xb = 2 * x - xo
    return x


@pytest.mark.slow
def test_tv_wls_matches_chambolle_pock_optimum():
    n, m, nb = 8, 12, 12
    _, b, w = _small_problem(7, n, m, nb, noise=0.1)
    beta = 0.5
    a = P.dense_matrix(n, m, nb)
    xc = _chambolle_pock_tv_wls(a, b.ravel(), w.ravel(), beta, n, 40000)
    res, _ = AP.lowdose_solve(b, w, beta, n, 600)
    f_app = AP.cost_lowdose(res.x, b, w, beta)
    f_cp = AP.cost_lowdose(xc.reshape(n, n), b, w, beta)
    assert abs(f_app - f_cp) <= 1e-7 * f_cp
    np.testing.assert_allclose(res.x.ravel(), xc, atol=2e-5)
    # saddle point: the partial gap 1/2 ||W^1/2 (Ax - b) - W^-1/2 mu||^2 vanishes
    assert AP.partial_gap(res.x, res.mu, b, w) < 1e-16 * f_app
    # and the primal step is a fixed point: x = prox(x - tau A^T mu; tau beta)
    st = AP.steps_lowdose(w, n)
    xf, _, _ = T.tv_prox(res.x - st.tau * P.back_project(res.mu, n), st.tau * beta, n_iter=20000)
    np.testing.assert_allclose(xf, res.x, atol=1e-7)


def test_cost_at_zero_image():
    rng = np.random.default_rng(1)
    b = rng.standard_normal((5, 9))
    w = rng.uniform(1, 2, (5, 9))
    assert AP.cost_lowdose(np.zeros((6, 6)), b, w, 0.7) == pytest.approx(0.5 * float((w * b * b).sum()))


def test_rmse_definition():
    x = np.full((4, 4), 2.0)
    assert AP.rmse(x, x - 0.25) == pytest.approx(0.25)
    assert AP.rmse(x, x) == 0.0


@pytest.mark.parametrize("winv", [True, False])
def test_simplified_extrapolation_equals_defining_form(winv):
    n, m, nb = 8, 12, 12
    _, b, w = _small_problem(3, n, m, nb)
    h = F.smoothed_ramp_taps(nb, m, 0.2, 0.5) if winv else F.ramp_taps(nb, m, 0.2)
    kw = dict(winv=1.0 / w) if winv else {}
    r1 = AP.app_solve(b, n, 6, 0.2, 0.3, h, beta=0.3, **kw)
    r2 = AP.app_solve(b, n, 6, 0.2, 0.3, h, beta=0.3, extrapolation="direct", **kw)
    np.testing.assert_allclose(r1.x, r2.x, atol=1e-12)
    np.testing.assert_allclose(r1.mu, r2.mu, atol=1e-12)


def test_first_iterate_is_filtered_backprojection_then_prox():
    # x^1 = prox(sigma tau A^T D b): with the ramp D(tau) = D(1)/tau this is
    # prox(sigma * FBP(b)) whatever tau is (Sec. 3 remark after Eq. 32).
    n, m, nb = 12, 16, 18
    _, b, _ = _small_problem(9, n, m, nb)
    tau, sigma = 0.37, 0.5
    res = AP.app_solve(b, n, 1, tau, sigma, F.ramp_taps(nb, m, tau), beta=1.0)
    fbp = P.back_project(F.apply_filter(b, F.ramp_taps(nb, m, 1.0)), n)
    ref, _, _ = T.tv_prox(sigma * fbp, tau)
    np.testing.assert_allclose(res.x, ref, atol=1e-12)


@pytest.mark.slow
def test_fewview_reaches_consistent_data():
    n, m, nb = 16, 6, 24
    xt = np.zeros((n, n))
    xt[4:12, 5:11] = 1.0
    xt[7:10, 2:6] = 0.5
    b = P.forward_project(xt, m, nb)
    res, st = AP.fewview_solve(b, n, 3000)
    assert AP.data_residual(res.x, b) < 1e-5
    assert res.x.min() >= 0.0
    assert T.tv_norm(res.x) <= T.tv_norm(xt) * (1 + 1e-4)


def test_lambda_max_matches_dense_eigendecomposition():
    n, m, nb = 10, 9, 14
    h = F.smoothed_ramp_taps(nb, m, 0.3, 0.2)
    op = lambda v: P.back_project(F.apply_filter(P.forward_project(v.reshape(n, n), m, nb), h), n).ravel()
    dense = AP.lambda_max(op, n * n)                  # dense eigvalsh path
    iterative = AP.lambda_max(op, n * n, dense_below=0)   # ARPACK path
    assert iterative == pytest.approx(dense, rel=1e-10)
    a = P.dense_matrix(n, m, nb)
    d = np.kron(np.eye(m), F.toeplitz_matrix(h))
    assert dense == pytest.approx(np.linalg.eigvalsh(a.T @ d @ a)[-1], rel=1e-12)


def test_step_sizes_satisfy_the_bounds():
    n, m, nb = 8, 12, 12
    _, b, w = _small_problem(11, n, m, nb)
    st = AP.steps_lowdose(w, n)
    winv = 1.0 / w
    h = F.smoothed_ramp_taps(nb, m, st.tau, float(winv.mean()))
    a = P.dense_matrix(n, m, nb)
    d = np.kron(np.eye(m), F.toeplitz_matrix(h))
    lam_a = np.linalg.eigvalsh(a.T @ d @ a)[-1]
    sw = np.sqrt(winv).ravel()
    lam_h = np.linalg.eigvalsh(sw[:, None] * d * sw[None, :])[-1]
    assert st.sigma < 2.0 / lam_h and st.tau * st.sigma * lam_a < 1.0
    assert max(st.sigma * lam_h / 2.0, st.tau * st.sigma * lam_a) == pytest.approx(0.95, rel=1e-9)
    sf = AP.steps_fewview(b, n)
    d1 = np.kron(np.eye(m), F.toeplitz_matrix(F.ramp_taps(nb, m, sf.tau)))
    assert sf.sigma * sf.tau * np.linalg.eigvalsh(a.T @ d1 @ a)[-1] == pytest.approx(0.95, rel=1e-9)


def test_identity_taps_apply_the_identity():
    rng = np.random.default_rng(7)
    s = rng.standard_normal((5, 9))
    np.testing.assert_array_equal(F.apply_filter(s, AP.identity_taps(9)), s)


def test_identity_steps_closed_forms():
    # lambda_h of W^-1/2 I W^-1/2 by the generic eigen-solver equals max 1/w;
    # lambda_A equals the dense largest eigenvalue of A^T A; the default tau
    # makes both bounds on sigma equal
    n, m, nb = 8, 12, 12
    _, b, w = _small_problem(3, n, m, nb)
    st = AP.steps_lowdose_identity(w, n)
    assert AP.lambda_h(1.0 / w, AP.identity_taps(nb)) == pytest.approx(st.lambda_h, rel=1e-10)
    a = P.dense_matrix(n, m, nb)
    assert st.lambda_a == pytest.approx(np.linalg.eigvalsh(a.T @ a)[-1], rel=1e-10)
    assert 2.0 / st.lambda_h == pytest.approx(1.0 / (st.tau * st.lambda_a), rel=1e-12)
    assert st.sigma == pytest.approx(0.95 * 2.0 / st.lambda_h, rel=1e-12)


def test_identity_solve_converges_to_nnls():
    # without the preconditioner the same iteration still solves Eq. 1 (beta = 0:
    # weighted NNLS), only more slowly: 4e-5 after 20000 iterations (1e-10 after
    # 50000) where Algorithm 1' is within 1e-9 after 1500
    n, m, nb = 8, 12, 12
    _, b, w = _small_problem(5, n, m, nb)
    a = P.dense_matrix(n, m, nb)
    sw = np.sqrt(w).ravel()
    ref, _ = nnls(sw[:, None] * a, sw * b.ravel())
    res, st = AP.lowdose_identity_solve(b, w, 0.0, n, 20000)
    np.testing.assert_allclose(res.x.ravel(), ref, atol=1e-4)
    res2, _ = AP.lowdose_identity_solve(b, w, 0.0, n, 10000)
    assert np.abs(res.x.ravel() - ref).max() < 0.1 * np.abs(res2.x.ravel() - ref).max()
