"""Pins of the oracle's error-tolerant few-view solver (the problem the
conclusions name: min psi(x) s.t. ||Ax - b|| <= eps, x >= 0), which the paper
only states:

* eps = 0 reproduces Algorithm 2 (a different oracle function) iterate for
  iterate;
* the ball projection against its closed form;
* the step-size norm lambda_max(K^T D K), K = [A, -I], against the dense
  matrix built from the dense system matrix and the Toeplitz filter;
* the limit: the same optimum (psi and x) as an independent Chambolle-Pock
  solve of the same problem, with the constraint active (||Ax - b|| = eps),
  x >= 0, and the fixed-point (KKT) relations of the iteration;
* eps >= ||b|| makes x = 0 feasible, so psi* = 0: the iterates' TV goes to zero.
"""
import numpy as np
import pytest
from scipy.linalg import toeplitz

from oracle import app as OA
from oracle import comparators as OC
from oracle import filters as OF
from oracle import projector as OP
from oracle import tv as OT
from paper_1609_06041_amd import synth as S


def small_problem(n=16, m=8, nb=24, seed=3):
    prob = S.make_problem(99, seed, n, m, nb, 4, None, with_x_true=True)
    return np.asarray(prob.b, np.float64), prob.x_true


def test_eps_zero_is_algorithm_2():
    n, m, nb = 20, 10, 30
    b, _ = small_problem(n, m, nb)
    st = OA.steps_fewview(b, n)
    ref, _ = OA.fewview_solve(b, n, 15, tau=st.tau, sigma=st.sigma)
    res, _ = OA.fewview_eps_solve(b, n, 0.0, 15, tau=st.tau, sigma=st.sigma)
    np.testing.assert_allclose(res.x, ref.x, rtol=0, atol=1e-13 * np.abs(ref.x).max())
    np.testing.assert_allclose(res.mu, ref.mu, rtol=0, atol=1e-13 * np.abs(ref.mu).max())
    np.testing.assert_array_equal(res.y, b)


def test_ball_projection_closed_form():
    rng = np.random.default_rng(0)
    b = rng.standard_normal((4, 5))
    d = rng.standard_normal((4, 5))
    inside = b + 0.5 * d / np.linalg.norm(d)
    np.testing.assert_array_equal(OA.ball_projection(inside, b, 1.0), inside)
    out = OA.ball_projection(b + 3.0 * d / np.linalg.norm(d), b, 1.0)
    assert np.linalg.norm(out - b) == pytest.approx(1.0, rel=1e-14)
    np.testing.assert_allclose((out - b) / np.linalg.norm(out - b), d / np.linalg.norm(d), rtol=1e-13)
    np.testing.assert_array_equal(OA.ball_projection(b + d, b, 0.0), b)


def test_split_norm_equals_dense_eigenvalue():
    n, m, nb = 6, 5, 9
    tau = 0.7
    h = OF.ramp_taps(nb, m, tau)
    A = OP.dense_matrix(n, m, nb)
    T = np.kron(np.eye(m), toeplitz(h[nb - 1:]))   # view-major sinogram, one Toeplitz block per view
    K = np.hstack([A, -np.eye(m * nb)])
    dense = np.linalg.eigvalsh(K.T @ T @ K)[-1]
    assert OA.lambda_a_split(n, m, nb, h) == pytest.approx(dense, rel=1e-10)


def test_converges_to_the_chambolle_pock_optimum():
    n, m, nb = 16, 8, 24
    b, _ = small_problem(n, m, nb)
    eps = 0.2 * np.linalg.norm(b)
    st = OA.steps_fewview_eps(b, n)
    res, _ = OA.fewview_eps_solve(b, n, eps, 3000, tau=st.tau, sigma=st.sigma, n_tv=20)
    cst = OC.cp_steps(n, m, nb)
    xc, _, _ = OC.cp_fewview_eps(b, n, eps, 20000, cst.dual, cst.primal)
    r = np.linalg.norm(OP.forward_project(res.x, m, nb) - b)
    rc = np.linalg.norm(OP.forward_project(xc, m, nb) - b)
    assert r == pytest.approx(eps, rel=2e-3)          # the constraint is active ...
    assert rc == pytest.approx(eps, rel=2e-3)
    # ... at the optimum: Chambolle-Pock approaches it slowly from above (2.8e-3 relative
    # after 20000 iterations, 2.5e-4 after 80000), so the APP value must lie below
    # its value and close to it, and the images agree
    psi, psic = OT.tv_norm(res.x), OT.tv_norm(xc)
    assert psic * (1.0 - 5e-3) <= psi <= psic * (1.0 + 1e-6)
    assert np.linalg.norm(res.x - xc) <= 2e-2 * np.linalg.norm(xc)
    assert res.x.min() >= 0.0
    # fixed point of the iteration: A x = y, y = P_B(y + tau mu), x = prox(x - tau A^T mu)
    assert np.linalg.norm(OP.forward_project(res.x, m, nb) - res.y) <= 1e-3 * np.linalg.norm(b)
    yy = OA.ball_projection(res.y + st.tau * res.mu, b, eps)
    assert np.linalg.norm(yy - res.y) <= 1e-3 * np.linalg.norm(b)
    xx, _, _ = OT.tv_prox(res.x - st.tau * OP.back_project(res.mu, n), st.tau, res.p1.copy(), res.p2.copy(), 200)
    assert np.linalg.norm(xx - res.x) <= 1e-3 * np.linalg.norm(res.x)


def test_eps_beyond_the_data_norm_reaches_zero_tv():
    # x = 0 is feasible, so psi* = 0; every feasible constant image c >= 0 is a
    # minimiser too, and the iterates settle on one of them
    n, m, nb = 12, 6, 18
    b, _ = small_problem(n, m, nb, seed=5)
    eps = 1.01 * np.linalg.norm(b)
    res, _ = OA.fewview_eps_solve(b, n, eps, 3000)
    first, _ = OA.fewview_eps_solve(b, n, eps, 1)
    assert OT.tv_norm(res.x) <= 1e-3 * OT.tv_norm(first.x)
    assert np.linalg.norm(OP.forward_project(res.x, m, nb) - b) <= eps
    assert res.x.min() >= 0.0
